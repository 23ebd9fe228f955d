"""Learned surrogate of one convection step (deep, then shallow on the updated state).

The network (include/mlp.h) maps the column's temperature, humidity and pressure on every level to
the step's total heating, moistening and precipitation.  Training pairs come from the FP64 scheme
itself: seeded synthetic soundings (``soundings``) are stepped by ``conv_step`` on the GPU, packed
and normalised by the library's kernels, and the network is trained by the library's BF16-MFMA
forward, backward, loss and Adam kernels.  Inference (``surr_infer``) falls back to the FP64 scheme
for columns whose predicted precipitation leaves the range seen in training.

This module is host-side control only: every computation on the path runs in libconv's kernels.
Torch supplies device memory, streams and the evaluation statistics.
"""
from __future__ import annotations

import ctypes as C
import math
import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np

from . import binding as B
from . import soundings as S

NLEV = 30
N_IN, N_OUT = 3 * NLEV, 2 * NLEV + 1
WIDTHS = (96, 512, 512, 512, 512, 64)
WARM_FRAC = 42.0 / 192.0  # tropical share of the 288 x 192 grid's rows (|lat| < 20 deg)


def _check(rc, what):
    B.check(rc, what)


def _state_struct(torch, dev, ncol):
    return B.state_struct(torch, dev, NLEV, ncol)


def generate(torch, n: int, seed0: int, chunk: int = 250_000, threads: int = 8, log=None):
    """n labelled soundings: raw float32 input rows X [n][96] and target rows Y [n][64] on the
    device.  Soundings of the 1-degree grid's distribution with the warm (tropical) recipe drawn
    independently per column with the grid's tropical share, so any contiguous slice is a fair
    sample; chunk i uses seed seed0 + i.  Returns (X, Y, seconds)."""
    t0 = time.perf_counter()
    L = B.lib()
    X = torch.empty(n, WIDTHS[0], dtype=torch.float32, device="cuda")
    Y = torch.empty(n, WIDTHS[-1], dtype=torch.float32, device="cuda")
    conv = B.Conv(chunk, NLEV)
    deep = conv.alloc_deep(chunk)
    shallow = conv.alloc_shallow(chunk)
    nchunks = (n + chunk - 1) // chunk

    def make(i):
        m = min(chunk, n - i * chunk)
        warm = np.random.default_rng(seed0 + i).random(m) < WARM_FRAC
        return S.make_state(m, NLEV, seed=seed0 + i, warm=warm)

    with ThreadPoolExecutor(max_workers=threads) as pool:
        futs = [pool.submit(make, i) for i in range(nchunks)]
        for i, f in enumerate(futs):
            st = f.result()
            m = st["ncol"]
            dev = B.to_device(st)
            if m == chunk:
                c, dd, ss = conv, deep, shallow
            else:  # the last, shorter chunk: its own context and outputs of leading dimension m
                c = B.Conv(m, NLEV)
                dd, ss = c.alloc_deep(m), c.alloc_shallow(m)
            c.step(dev, dd, ss)
            sst = _state_struct(torch, dev, m)
            _check(L.surr_pack_inputs_raw(C.byref(sst), NLEV, m, WIDTHS[0],
                                          C.c_void_p(X[i * chunk].data_ptr()), B._stream(torch)),
                   "surr_pack_inputs_raw")
            d, s = B.Conv._deep_struct(dd), B.Conv._shallow_struct(ss)
            _check(L.surr_pack_targets_raw(C.byref(d), C.byref(s), NLEV, m, m, WIDTHS[-1],
                                           C.c_void_p(Y[i * chunk].data_ptr()), B._stream(torch)),
                   "surr_pack_targets_raw")
            futs[i] = None
            if log and (i + 1) % 10 == 0:
                log(f"generated {min((i + 1) * chunk, n)} / {n}")
    torch.cuda.synchronize()
    return X, Y, time.perf_counter() - t0


def col_stats(torch, a, n_valid):
    """(mean, std, rms) per feature of a [n][w] (surr_col_stats)."""
    L = B.lib()
    w = a.shape[1]
    mean, std, rms = (torch.empty(w, dtype=torch.float32, device="cuda") for _ in range(3))
    nb = L.surr_col_stats_scratch_bytes(w)
    scratch = torch.empty(nb, dtype=torch.uint8, device="cuda")
    _check(L.surr_col_stats(C.c_void_p(a.data_ptr()), a.shape[0], w, n_valid,
                            C.c_void_p(mean.data_ptr()), C.c_void_p(std.data_ptr()),
                            C.c_void_p(rms.data_ptr()), C.c_void_p(scratch.data_ptr()), nb,
                            B._stream(torch)), "surr_col_stats")
    return mean, std, rms


def normalize(torch, a, mean, std, to_bf16: bool):
    """(a - mean) / std: a new bfloat16 tensor, or in place."""
    L = B.lib()
    out = torch.empty(a.shape, dtype=torch.bfloat16, device="cuda") if to_bf16 else None
    _check(L.surr_normalize(C.c_void_p(a.data_ptr()), a.shape[0], a.shape[1],
                            C.c_void_p(mean.data_ptr()), C.c_void_p(std.data_ptr()),
                            None if out is None else C.c_void_p(out.data_ptr()), B._stream(torch)),
           "surr_normalize")
    return out if to_bf16 else a


def group_scales(torch, rms):
    """Target normalisation by output group: mean 0 and, for every level of the heating and of the
    moistening profile and for the precipitation, one scale = the group's root-mean-square.  Per-
    level statistics would divide the rare tendencies of levels that convection seldom reaches by a
    tiny spread and let those outliers dominate the loss."""
    ms = rms.double() ** 2
    scale = torch.ones_like(rms)
    for a, b in ((0, NLEV), (NLEV, 2 * NLEV), (2 * NLEV, N_OUT)):
        scale[a:b] = float(torch.sqrt(ms[a:b].mean()))
    return torch.zeros_like(rms), scale


def init_params(torch, seed: int):
    """W ~ N(0, 1/fan_in) (the usual variance-preserving start for GELU layers), b = 0."""
    g = torch.Generator(device="cpu").manual_seed(seed)
    parts = []
    for i in range(len(WIDTHS) - 1):
        parts.append((torch.randn(WIDTHS[i + 1], WIDTHS[i], generator=g) / math.sqrt(WIDTHS[i])).reshape(-1))
        parts.append(torch.zeros(WIDTHS[i + 1]))
    return torch.cat(parts).to(torch.float32)


def train(torch, net, Xb, Yn, epochs: int, batch: int, lr: float, seed: int = 0, log=None):
    """Adam over `epochs` passes of contiguous minibatches in a random order per epoch, with a
    cosine-decayed learning rate.  Returns (per-epoch mean loss, seconds, steps)."""
    n = Xb.shape[0]
    nb = n // batch
    steps = epochs * nb
    hist = torch.zeros(steps, dtype=torch.float32, device="cuda")
    rng = np.random.default_rng(seed)
    t0 = time.perf_counter()
    k = 0
    y = torch.empty(batch, WIDTHS[-1], dtype=torch.float32, device="cuda")
    for ep in range(epochs):
        for b in rng.permutation(nb):
            sl = slice(int(b) * batch, int(b + 1) * batch)
            a = 0.5 * (1.0 + math.cos(math.pi * k / steps))
            net.train_step(Xb[sl], Yn[sl], N_OUT, lr * (0.02 + 0.98 * a), y=y, loss=hist[k:k + 1])
            k += 1
        if log:
            torch.cuda.synchronize()
            log(f"epoch {ep + 1}/{epochs}: loss {hist[k - nb:k].mean().item():.5f}")
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    per_epoch = hist.view(epochs, nb).mean(dim=1).cpu().tolist()
    return per_epoch, secs, steps


class Surrogate:
    """Trained network + normalisation + fallback range, applied through surr_infer."""

    def __init__(self, net, norms, prec_range, max_cols: int, chunk: int, params=None):
        torch = net.torch
        self.torch, self.net = torch, net
        L = B.lib()
        self.params = params or B.make_params()
        nbytes = L.surr_workspace_bytes(NLEV, WIDTHS[0], WIDTHS[-1], max_cols, chunk)
        if nbytes == 0:
            raise ValueError("unsupported surrogate size")
        self.ws = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
        h = C.c_void_p()
        _check(L.surr_create(net.h, NLEV, WIDTHS[0], WIDTHS[-1], max_cols, chunk,
                             C.byref(self.params), C.c_void_p((self.ws.data_ptr() + 255) & ~255),
                             nbytes, C.byref(h)), "surr_create")
        self.h = h
        self.max_cols = max_cols
        in_mean, in_std, out_mean, out_std = norms
        self.norms = norms
        self.prec_range = prec_range
        _check(L.surr_set_norm(h, *[C.c_void_p(t.data_ptr()) for t in (in_mean, in_std, out_mean,
                                                                         out_std)],
                               float(prec_range[0]), float(prec_range[1]), B._stream(torch)),
               "surr_set_norm")

    def __del__(self):
        try:
            if getattr(self, "h", None):
                B.lib().surr_destroy(self.h)
                self.h = None
        except Exception:
            pass

    def set_fused(self, enable: bool) -> bool:
        """Choose the fused inference kernel (default) or the layer-by-layer path; returns whether
        the next inference takes the fused kernel."""
        rc = B.lib().surr_set_fused(self.h, int(enable))
        _check(min(rc, 0), "surr_set_fused")
        return rc == 1

    def infer(self, dev, ncol: int, fallback: bool = True, out=None):
        """Returns (dTdt [L][ld], dqdt [L][ld], prec [ld], n_fallback or None)."""
        torch = self.torch
        ld = dev["T"].shape[1]
        if out is None:
            out = (torch.empty(NLEV, ld, dtype=torch.float64, device="cuda"),
                   torch.empty(NLEV, ld, dtype=torch.float64, device="cuda"),
                   torch.empty(ld, dtype=torch.float64, device="cuda"))
        st = _state_struct(torch, dev, ncol)
        nfb = C.c_int64(-1)
        _check(B.lib().surr_infer(self.h, C.byref(st), ncol, *[C.c_void_p(t.data_ptr()) for t in out],
                                  int(fallback), C.byref(nfb), B._stream(torch)), "surr_infer")
        return out[0], out[1], out[2], (nfb.value if fallback else None)


def errors(torch, pred, deep, shallow, ncol):
    """Error of predicted total tendencies against the FP64 scheme's, per output: RMSE, the RMS of
    the truth, their ratio, and the same over convecting columns only."""
    dT, dq, pr = pred
    tT = (deep["dTdt"] + shallow["dTdt"])[:, :ncol]
    tq = (deep["dqdt"] + shallow["dqdt"])[:, :ncol]
    tp = (deep["prec"] + shallow["prec"])[:ncol]
    act = (deep["status"][:ncol] == 0) | (shallow["status"][:ncol] == 0)
    out = {}
    for name, p, t, cols in (("dTdt", dT[:, :ncol], tT, 1), ("dqdt", dq[:, :ncol], tq, 1),
                             ("prec", pr[:ncol], tp, 0)):
        e = p - t
        rmse = float(torch.sqrt((e ** 2).mean()))
        rms = float(torch.sqrt((t ** 2).mean()))
        ea = e[..., act] if cols else e[act]
        ta = t[..., act] if cols else t[act]
        out[name] = {"rmse": rmse, "rms_truth": rms, "rel_rmse": rmse / rms if rms > 0 else None,
                     "rel_rmse_convecting": float(torch.sqrt((ea ** 2).mean()) /
                                                  torch.sqrt((ta ** 2).mean()))}
    out["convecting_fraction"] = float(act.double().mean())
    return out


def build_and_train(torch, n_train: int, epochs: int, batch: int = 16384, lr: float = 1e-3,
                    seed: int = 105, log=None, max_cols: int = 884_736, chunk: int = 131_072):
    """Generate, normalise, train; returns (Surrogate, report dict).  n_train + 100,000 soundings
    are generated; the last 100,000 are held out."""
    hold = 100_000
    X, Y, gen_s = generate(torch, n_train + hold, seed * 1000, log=log)
    in_mean, in_std, _ = col_stats(torch, X[:n_train], N_IN)
    out_mean, out_std = group_scales(torch, col_stats(torch, Y[:n_train], N_OUT)[2])
    prec_max = float(Y[:n_train, N_OUT - 1].max())
    Xb = normalize(torch, X, in_mean, in_std, to_bf16=True)
    del X
    Yn = normalize(torch, Y, out_mean, out_std, to_bf16=False)
    net = B.MLP(WIDTHS, max_batch=max(batch, chunk, hold), max_train_batch=batch)
    net.set_params(init_params(torch, seed).cuda())
    curve, train_s, steps = train(torch, net, Xb[:n_train], Yn[:n_train], epochs, batch, lr,
                                  seed=seed, log=log)
    yh = net.forward(Xb[n_train:], keep=False)
    hold_loss = float(net.mse(yh, Yn[n_train:], N_OUT).item())
    flops = 3 * 2 * sum(WIDTHS[i] * WIDTHS[i + 1] for i in range(len(WIDTHS) - 1)) * steps * batch
    report = {"n_train": n_train, "n_holdout": hold, "epochs": epochs, "batch": batch, "lr": lr,
              "generate_s": gen_s, "train_s": train_s, "train_steps": steps,
              "train_TFLOPs": flops / train_s / 1e12, "loss_per_epoch": curve,
              "holdout_loss": hold_loss, "prec_max_train": prec_max}
    sur = Surrogate(net, (in_mean, in_std, out_mean, out_std),
                    (-0.05 * prec_max, prec_max), max_cols, chunk)
    return sur, report
