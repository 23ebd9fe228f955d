#!/usr/bin/env python3
"""Benchmark: one physics step of FP64 deep + shallow convection (the paper's Algorithm 1 order)
over the 1152 x 768 = 884,736-column x 30-level latitude-clustered synthetic grid on one MI355X.

Prints ONE JSON line.  `value` is columns per second of the whole step with inputs resident in HBM.
`roofline` is for the kernel that takes the most time in the step, its duration measured live with
HIP events recorded by the library on the stream it launches on.  `cpu_baseline` is the CPU oracle
(OpenMP dynamic schedule over the host cores, the paper's own load-balancing technique) timed on
the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("convection columns/s (FP64, 1 GPU) at 884,736×30; adjoint/forward cost; "
          "surrogate error")
HBM_PEAK_GBS = 8000.0
NLEV = 30
NLON, NLAT = 1152, 768


# HBM traffic per launch measured with rocprofv3 on the 884,736 x 30 step (FETCH_SIZE and
# WRITE_SIZE in KiB per dispatch, scaled by what a plain 1 GiB copy kernel reads on the same
# counters: x2.0 and x1.0; profiles/conv_step_884736x30_hbm_traffic.md).  Valid only while the
# kernel sources hash to `sources_sha256`; otherwise `traffic` is reported as null.
TRAFFIC_SOURCES = ("paper_1711_00289_amd/csrc/conv.hip", "paper_1711_00289_amd/csrc/conv_physics.hpp",
                   "paper_1711_00289_amd/csrc/conv_internal.hpp")
MEASURED_TRAFFIC = {
    "sources_sha256": "1481265f74d2f85489f797ac30f13960c3ec85057cc002f60663154ff552dd3f",
    "fetch_factor": 2.0, "write_factor": 1.0,
    "k_trigger": (542324, 1530011),
    "k_deep_plume": (143573, 183520),
    "k_shallow_retrigger": (164584, 25922),
}


def measured_traffic(kernel: str):
    """Calibrated HBM bytes per launch of `kernel`, or None if the sources changed since."""
    import hashlib

    h = hashlib.sha256()
    for p in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    m = MEASURED_TRAFFIC
    if h.hexdigest() != m["sources_sha256"] or kernel not in m:
        return None
    fetch, write = m[kernel]
    return int((fetch * m["fetch_factor"] + write * m["write_factor"]) * 1024)


def bytes_per_column(L: int):
    """Algorithmic HBM bytes per column of the fused step: every input read once, every output
    written once."""
    inputs = (4 * L + (L + 1) + 3) * 8
    deep_scalars = 8 + 4 * 4                         # cape, klaunch, ktop, trig, status
    deep_arrays = (2 * L + 2 * (L + 1) + 1) * 8      # dTdt, dqdt, mu, md, prec
    shallow = (2 * L + (L + 1) + 2) * 8 + 3 * 4     # dTdt, dqdt, mu, prec, cin, kbase, ktop, status
    return dict(inputs=inputs, deep_scalars=deep_scalars, deep_arrays=deep_arrays,
                shallow=shallow, total=inputs + deep_scalars + deep_arrays + shallow)


def kernel_bytes(L, n, trig, sh_status):
    """Algorithmic bytes attributed to each kernel of the step (each input read and each output
    written once, charged to the kernel that does it).  The shallow plumes run inside the
    re-trigger kernel in the step (k_shallow_plume serves the shallow scheme alone)."""
    b = bytes_per_column(L)
    quiet = trig == 0
    sh_done = ~np.isin(sh_status, (0, 5))
    return dict(
        trigger=int(n * (b["inputs"] + b["deep_scalars"]) + quiet.sum() * b["deep_arrays"] +
                    (quiet & sh_done).sum() * b["shallow"]),
        deep_plume=int((~quiet).sum() * b["deep_arrays"]),
        shallow_retrigger=int((((~quiet) & sh_done) | ~sh_done).sum() * b["shallow"]),
        shallow_plume=0,
        reset=0,
    )


OMP_CHUNKS = (1, 2, 4, 8, 14, 16)


def cpu_baseline(st, threads, chunk=16, min_cpu_s=15.0, max_steps=20):
    """The oracle's step over the whole grid on `threads` host threads (OpenMP dynamic schedule,
    `chunk` columns per grab), repeated until about `min_cpu_s` thread-seconds of work have run
    (bounded by `max_steps`)."""
    import oracle

    steps = 0
    t0 = time.perf_counter()
    while True:
        oracle.step(st, threads=threads, chunk=chunk)
        steps += 1
        dt = time.perf_counter() - t0
        if dt * threads >= min_cpu_s or steps >= max_steps:
            break
    return steps * st["ncol"] / dt, dt, steps


def cpu_model():
    """The host CPU's model name (lscpu), or None."""
    import subprocess

    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
    except (OSError, subprocess.SubprocessError):
        return None
    for line in out.splitlines():
        if line.startswith("Model name:"):
            return line.split(":", 1)[1].strip()
    return None


def oracle_ops(st, stride=16):
    """The oracle's algorithmic operation count of the step (+, -, *, /, sqrt, exp, log = 1 each)
    per column, averaged over every `stride`-th column of the grid."""
    import oracle
    from paper_1711_00289_amd import soundings as S

    sub = S.subset(st, list(range(0, st["ncol"], stride)))
    return float(oracle.step_ops(sub).mean()), sub["ncol"]


def cpu_one_thread(st, stride=1):
    """The plain single-threaded oracle step over every `stride`-th column of the grid (the whole
    grid by default: a few seconds on one core)."""
    import oracle
    from paper_1711_00289_amd import soundings as S

    sub = st if stride == 1 else S.subset(st, list(range(0, st["ncol"], stride)))
    t0 = time.perf_counter()
    oracle.step(sub)
    dt = time.perf_counter() - t0
    return sub["ncol"] / dt, dt, sub["ncol"]


def copy_bandwidth(torch, mib=1024, reps=5):
    """GB/s (bytes read + written) of a plain device-to-device copy of `mib` MiB: the practical
    ceiling the step's HBM fraction is compared with."""
    nb = mib * (1 << 20)
    src = torch.ones(nb // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    ms = time_events(torch, lambda: dst.copy_(src), reps)
    del src, dst
    return 2 * nb / (ms * 1e-3) / 1e9


def time_events(torch, fn, reps, stream=None):
    """Average ms of `fn()` over `reps` calls, bracketed by events on `stream` (default: current)."""
    stream = stream or torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(reps):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def adjoint_bytes(L: int, n: int, nact: int) -> int:
    """Algorithmic HBM bytes of one conv_deep_backward call (cotangents of dTdt and dqdt, none of
    prec): every column reads its status and writes g_T and g_q; an active column also reads its
    inputs T, q, p_mid, z, p_int and phis, its launch and top levels and both cotangents."""
    quiet = 4 + 2 * L * 8
    active = (4 * L + (L + 1) + 1) * 8 + 2 * 4 + 2 * L * 8
    return n * quiet + nact * active


def bench_adjoint(torch, B, S, reps):
    """Deep forward and hand-written adjoint on the 288x192 = 55,296-column x 30-level grid with the
    loss sum(a*dTdt^2 + b*(Lv/cp*dqdt)^2), a, b ~ N(0,1)."""
    st = S.grid_1deg(NLEV)
    n = st["ncol"]
    dev = B.to_device(st)
    conv = B.Conv(n, NLEV)
    out = conv.deep_forward(dev)
    g = torch.Generator(device="cpu").manual_seed(4)
    a = torch.randn(NLEV, n, generator=g, dtype=torch.float64).cuda()
    b = torch.randn(NLEV, n, generator=g, dtype=torch.float64).cuda()
    lvcp = 2.501e6 / 1004.64
    cT = 2.0 * a * out["dTdt"]
    cq = 2.0 * b * lvcp ** 2 * out["dqdt"]
    for _ in range(3):
        conv.deep_forward(dev, out)
        conv.deep_backward(dev, out, cT, cq, None)
    fwd = time_events(torch, lambda: conv.deep_forward(dev, out), reps)
    bwd = time_events(torch, lambda: conv.deep_backward(dev, out, cT, cq, None), reps)
    # The whole step (deep, update, shallow) and its adjoint, with the same loss on the deep and
    # the shallow tendencies.
    deep, shallow = conv.step(dev)
    dcot = (2.0 * a * deep["dTdt"], 2.0 * b * lvcp ** 2 * deep["dqdt"], None)
    scot = (2.0 * a * shallow["dTdt"], 2.0 * b * lvcp ** 2 * shallow["dqdt"], None)
    for _ in range(3):
        conv.step(dev, deep, shallow)
        conv.step_backward(dev, deep, shallow, dcot, scot)
    sfwd = time_events(torch, lambda: conv.step(dev, deep, shallow), reps)
    sbwd = time_events(torch, lambda: conv.step_backward(dev, deep, shallow, dcot, scot), reps)
    nact = int((out["status"] == 0).sum())
    abytes = adjoint_bytes(NLEV, n, nact)
    return {"workload": "deep adjoint, 288x192 = 55,296 columns x 30 levels",
            "forward_ms": fwd, "backward_ms": bwd, "ratio": bwd / fwd,
            "active_fraction": nact / n,
            "roofline": {"bound": "hbm", "achieved": abytes / (bwd * 1e-3) / 1e9,
                         "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": abytes / (bwd * 1e-3) / 1e9 / HBM_PEAK_GBS,
                         "algorithmic_bytes_per_call": abytes,
                         "adjoint_wavefronts": 4 * -(-nact // 64),
                         "note": "four wavefronts per 64 active columns (updraft, two parcel halves, "
                                 "downdraft chains in parallel): the call is as long as the "
                                 "updraft's recompute-then-reverse chain"},
            "step": {"workload": "adjoint of the whole step (deep, update, shallow), same grid",
                     "forward_ms": sfwd, "backward_ms": sbwd, "ratio": sbwd / sfwd,
                     "shallow_active_fraction":
                         float((shallow["status"] == 0).double().mean())}}


NTRACERS = 8


def tracer_bytes(L, ntr, deep, shallow):
    """Algorithmic HBM bytes of one conv_tracer_transport call: the tendency written once for every
    column, the tracers read over the active plumes' levels, the plumes' mass fluxes, interface
    pressures and (shallow) heights, and the statuses of every column."""
    import numpy as np

    ds, ss = deep["status"], shallow["status"]
    n = ds.size
    total = ntr * L * 8 * n + 8 * n
    a = ds == 0
    kb, kt = deep["klaunch"][a].astype(np.int64), deep["ktop"][a].astype(np.int64)
    nl = kb - kt + 1                                     # layers kt .. kb
    total += int((ntr * nl * 8 + 2 * (nl - 1) * 8 + (nl + 1) * 8 + 8).sum())
    b = ss == 0
    ks, kts = shallow["kbase"][b].astype(np.int64), shallow["ktop"][b].astype(np.int64)
    nl = L - kts                                         # layers kts .. L-1
    total += int((ntr * nl * 8 + (ks - kts) * 8 + (nl + 1) * 8 + (ks - kts + 1) * 8 + 8).sum())
    return total


def bench_tracers(torch, B, conv, dev, deep, shallow, reps):
    """Convective transport of 8 passive tracers (exp of N(0,1), seeded) by the headline grid's
    step: time per call and the HBM roofline of k_tracers."""
    L, n = conv.nlev, conv.ncol
    g = torch.Generator(device="cuda").manual_seed(12)
    tr = torch.exp(torch.randn((NTRACERS, L, n), generator=g, dtype=torch.float64, device="cuda"))
    tend = torch.empty_like(tr)
    for _ in range(3):
        conv.tracer_transport(dev, deep, shallow, tr, out=tend)
    ms = time_events(torch, lambda: conv.tracer_transport(dev, deep, shallow, tr, out=tend), reps)
    host = lambda o: {k: o[k].cpu().numpy() for k in ("status", "klaunch", "ktop", "kbase")
                      if k in o}
    nbytes = tracer_bytes(L, NTRACERS, host(deep), host(shallow))
    achieved = nbytes / (ms * 1e-3) / 1e9
    return {"workload": f"{NTRACERS} passive tracers transported by the 884,736 x 30 step",
            "ms": ms, "columns_per_s": n / (ms * 1e-3),
            "roofline": {"bound": "hbm", "kernel": "k_tracers", "achieved": achieved,
                         "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                         "algorithmic_bytes_per_launch": nbytes}}


def bench_momentum(torch, B, conv, dev, deep, shallow, reps, c_pgf=0.7):
    """Convective momentum transport (u, v with the pressure-gradient term, coefficient c_pgf) by
    the headline grid's step: time per call and the HBM roofline of the transport kernel (the
    algorithmic bytes of two tracers)."""
    L, n = conv.nlev, conv.ncol
    g = torch.Generator(device="cuda").manual_seed(13)
    base = torch.linspace(25.0, -8.0, L, dtype=torch.float64, device="cuda")[:, None]
    w = torch.stack([base + 4.0 * torch.randn((L, n), generator=g, dtype=torch.float64,
                                              device="cuda"),
                     -0.4 * base + 4.0 * torch.randn((L, n), generator=g, dtype=torch.float64,
                                                     device="cuda")])
    tend = torch.empty_like(w)
    for _ in range(3):
        conv.momentum_transport(dev, deep, shallow, w, c_pgf=c_pgf, out=tend)
    ms = time_events(torch, lambda: conv.momentum_transport(dev, deep, shallow, w, c_pgf=c_pgf,
                                                            out=tend), reps)
    host = lambda o: {k: o[k].cpu().numpy() for k in ("status", "klaunch", "ktop", "kbase")
                      if k in o}
    nbytes = tracer_bytes(L, 2, host(deep), host(shallow))
    achieved = nbytes / (ms * 1e-3) / 1e9
    return {"workload": f"momentum (u, v) transported by the 884,736 x 30 step, c_pgf = {c_pgf}",
            "ms": ms, "columns_per_s": n / (ms * 1e-3),
            "roofline": {"bound": "hbm", "kernel": "k_tracers", "achieved": achieved,
                         "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                         "algorithmic_bytes_per_launch": nbytes}}


def bench_dilute(torch, B, dev, n, reps, eps_cape=1e-4):
    """The step on the headline grid with the dilute (entraining) CAPE parcel."""
    conv = B.Conv(n, NLEV, B.make_params(eps_cape=eps_cape))
    deep, shallow = conv.step(dev)
    for _ in range(3):
        conv.step(dev, deep, shallow)
    ms = time_events(torch, lambda: conv.step(dev, deep, shallow), reps)
    return {"workload": f"conv_step on the 884,736 x 30 grid with eps_cape = {eps_cape} 1/m",
            "ms_per_step": ms, "columns_per_s": n / (ms * 1e-3),
            "deep_active_fraction": float((deep["status"] == 0).double().mean()),
            "shallow_active_fraction": float((shallow["status"] == 0).double().mean())}


def bench_ensemble(torch, B, S, main_state, main_deep, main_shallow, reps, tune=True):
    """The 884,736-column grid plus 16 members of 55,296 columns (30/46/72 levels, tau 1800/3600/
    7200 s) as one ensemble: autotuned launch shape, captured HIP graph, timed replays; and the
    same members stepped one after the other for comparison."""
    members = [dict(state=main_state, nlev=NLEV, ncol=main_state["ncol"],
                    params=B.make_params(), deep=main_deep, shallow=main_shallow)]
    for m in range(16):
        sp = S.ensemble_member_spec(m)
        members.append(dict(state=B.to_device(S.ensemble_member(m)), nlev=sp["nlev"],
                            ncol=sp["ncol"], params=B.make_params(tau=sp["tau"])))
    ens = B.Ensemble(members)
    if tune:
        ens.autotune(reps=5)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    ens.capture(side)
    for _ in range(3):
        ens.replay(side)
    ms = time_events(torch, lambda: ens.replay(side), reps, stream=side)
    convs = [B.Conv(m["ncol"], m["nlev"], m["params"]) for m in ens.members]

    def separate():
        for c, m in zip(convs, ens.members):
            c.step(m["state"], m["deep"], m["shallow"])

    separate()
    sep = time_events(torch, separate, max(2, reps // 4))
    ncol = sum(m["ncol"] for m in ens.members)
    ebytes = sum(bytes_per_column(m["nlev"])["total"] * m["ncol"] for m in ens.members)
    return {"workload": "884,736x30 grid + 16 members x 55,296 columns (nlev 30/46/72, "
                        "tau 1800/3600/7200 s), one captured graph per step",
            "columns": ncol, "ms_per_step": ms, "columns_per_s": ncol / (ms * 1e-3),
            "roofline": {"bound": "hbm", "achieved": ebytes / (ms * 1e-3) / 1e9,
                         "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": ebytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                         "algorithmic_bytes_per_step": int(ebytes)},
            "launch_waves_per_cu": list(ens.get_launch()), "separate_calls_ms": sep,
            "batching_speedup": sep / ms}


def bench_surrogate(torch, B, main_state, truth_deep, truth_shallow, conv_step_ms, n_train, epochs,
                    reps):
    """Train the MLP surrogate on n_train soundings labelled by conv_step (plus 100,000 held out),
    then time its inference on the 884,736-column grid with and without the fallback to the scheme
    and measure its error against the scheme's tendencies on that grid."""
    from paper_1711_00289_amd import surrogate as SG

    n = main_state["ncol"]
    sur, rep = SG.build_and_train(torch, n_train, epochs, batch=16384, lr=1e-3, seed=105,
                                  max_cols=n, chunk=n,
                                  log=lambda m: print(f"[bench] surrogate {m}", file=sys.stderr,
                                                      flush=True))
    out = [torch.empty(NLEV, n, dtype=torch.float64, device="cuda") for _ in range(2)]
    out.append(torch.empty(n, dtype=torch.float64, device="cuda"))
    sur.infer(main_state, n, fallback=False, out=tuple(out))
    ms_nofb = time_events(torch, lambda: sur.infer(main_state, n, fallback=False, out=tuple(out)),
                          reps)
    nfb = sur.infer(main_state, n, fallback=True, out=tuple(out))[3]
    ms_fb = time_events(torch, lambda: sur.infer(main_state, n, fallback=True, out=tuple(out)), reps)
    err = SG.errors(torch, tuple(out), truth_deep, truth_shallow, n)
    flop_per_col = 2 * sum(SG.WIDTHS[i] * SG.WIDTHS[i + 1] for i in range(len(SG.WIDTHS) - 1))
    infer_tf = flop_per_col * n / (ms_nofb * 1e-3) / 1e12
    rep.pop("loss_per_epoch", None)
    return {"workload": f"MLP {SG.WIDTHS} GELU, BF16 operands / FP32 accumulation, trained on "
                        f"{n_train:,} soundings labelled by conv_step; inference on the "
                        f"884,736-column grid",
            "training": rep, "infer_ms": ms_nofb, "infer_with_fallback_ms": ms_fb,
            "fallback_columns": nfb, "conv_step_ms": conv_step_ms,
            "speedup_vs_scheme": conv_step_ms / ms_fb,
            "infer_TFLOPs": infer_tf,
            "mfma_roofline": {"bound": "mfma", "peak": 2500.0, "unit": "TFLOP/s",
                              "infer_frac": infer_tf / 2500.0,
                              "train_frac": rep["train_TFLOPs"] / 2500.0},
            "error_vs_scheme": err}


def bench_gemm(torch, B, reps, warmup):
    """The surrogate's hidden-layer product alone: C = GELU(A . W^T + b) with BF16 operands, FP32
    accumulation, BF16 output and the FP32 pre-activation kept, on random operands of
    M x 512 x 512 for M = 131,072 and 884,736."""
    g = torch.Generator(device="cuda").manual_seed(3)
    res = {"workload": "mlp_gemm_nt, bias + GELU, BF16 operands / FP32 accumulation, K = N = 512"}
    for M in (131072, 884736):
        a = torch.randn(M, 512, generator=g, device="cuda").to(torch.bfloat16)
        w = (torch.randn(512, 512, generator=g, device="cuda") / 512 ** 0.5).to(torch.bfloat16)
        b = torch.randn(512, generator=g, device="cuda")
        for _ in range(max(1, warmup)):
            B.gemm_nt(a, w, b, mode=1, z=True)
        ms = time_events(torch, lambda: B.gemm_nt(a, w, b, mode=1, z=True), reps)
        res[f"{M}x512x512"] = {"ms": ms, "TFLOPs": 2 * M * 512 * 512 / (ms * 1e-3) / 1e12}
        del a
    return res


def bench_infer_only(torch, B, reps, warmup):
    """Surrogate inference alone on the 884,736-column grid with a randomly initialised network
    (no training): time per call and the rate against the BF16 MFMA peak."""
    from paper_1711_00289_amd import soundings as S
    from paper_1711_00289_amd import surrogate as SG

    st = S.grid_quarter_deg(NLEV)
    n = st["ncol"]
    dev = B.to_device(st)
    net = B.MLP(SG.WIDTHS, max_batch=n, max_train_batch=4096)
    net.set_params(SG.init_params(torch, 1).cuda())
    f32 = lambda v: torch.tensor(v, dtype=torch.float32, device="cuda")
    norms = (f32(np.r_[np.full(NLEV, 250.0), np.full(NLEV, 5e-3), np.full(NLEV, 5e4),
                       np.zeros(SG.WIDTHS[0] - 3 * NLEV)]),
             f32(np.r_[np.full(NLEV, 20.0), np.full(NLEV, 5e-3), np.full(NLEV, 3e4),
                       np.ones(SG.WIDTHS[0] - 3 * NLEV)]),
             f32(np.zeros(SG.WIDTHS[-1])),
             f32(np.r_[np.full(NLEV, 1e-4), np.full(NLEV, 1e-7), [1e-4],
                       np.ones(SG.WIDTHS[-1] - 2 * NLEV - 1)]))
    sur = SG.Surrogate(net, norms, (-1.0, 1.0), n, n)
    out = tuple([torch.empty(NLEV, n, dtype=torch.float64, device="cuda") for _ in range(2)] +
                [torch.empty(n, dtype=torch.float64, device="cuda")])
    for _ in range(max(1, warmup)):
        sur.infer(dev, n, fallback=False, out=out)
    ms = time_events(torch, lambda: sur.infer(dev, n, fallback=False, out=out), reps)
    flop = 2 * sum(SG.WIDTHS[i] * SG.WIDTHS[i + 1] for i in range(len(SG.WIDTHS) - 1)) * n
    tf = flop / (ms * 1e-3) / 1e12
    # the layer-by-layer path (mlp_forward on the whole grid as one batch) for comparison
    sur.set_fused(False)
    sur.infer(dev, n, fallback=False, out=out)
    ms_lay = time_events(torch, lambda: sur.infer(dev, n, fallback=False, out=out), reps)
    sur.set_fused(True)
    return {"workload": f"surrogate inference, MLP {SG.WIDTHS} (random weights), 884,736 "
                        f"columns in one call", "ms": ms, "TFLOPs": tf,
            "mfma_frac": tf / 2500.0, "layer_by_layer_ms": ms_lay}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--ncol", type=int, default=NLON * NLAT)
    ap.add_argument("--launch", type=str, default="", help="deep,shallow plume wavefronts per CU")
    ap.add_argument("--no-tune", action="store_true", help="keep the default launch shape")
    ap.add_argument("--no-extras", action="store_true",
                    help="time only the headline step (no adjoint, ensemble)")
    ap.add_argument("--surrogate-n", type=int, default=10_000_000,
                    help="training soundings for the surrogate (0 skips it)")
    ap.add_argument("--surrogate-epochs", type=int, default=30)
    ap.add_argument("--gemm-only", action="store_true",
                    help="time only the surrogate's GEMM kernel (mlp_gemm_nt, bias + GELU) on "
                         "131,072 and 884,736 x 512 x 512 and exit")
    ap.add_argument("--infer-only", action="store_true",
                    help="time only the surrogate's inference (random network, no training) on "
                         "the 884,736-column grid and exit")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="after timing, copy a MIB-MiB device buffer once (a plain copy kernel of "
                         "known size for scaling hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}): the multi-GPU column "
              "sharding is designed but not built", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1711_00289_amd import binding as B
    from paper_1711_00289_amd import soundings as S

    if args.gemm_only:
        print(json.dumps(bench_gemm(torch, B, args.steps, args.warmup)), flush=True)
        return
    if args.infer_only:
        print(json.dumps(bench_infer_only(torch, B, args.steps, args.warmup)), flush=True)
        return

    t0 = time.perf_counter()
    if args.ncol == NLON * NLAT:
        st = S.grid_quarter_deg(NLEV)
    else:
        st = S.make_state(args.ncol, NLEV, seed=103,
                          warm=S.latlon_warm_mask(NLON, NLAT)[:args.ncol])
    n = st["ncol"]
    print(f"[bench] inputs generated ({n} columns) in {time.perf_counter() - t0:.1f} s",
          file=sys.stderr, flush=True)
    dev = B.to_device(st)
    conv = B.Conv(n, NLEV)
    deep = conv.alloc_deep(n)
    shallow = conv.alloc_shallow(n)
    if args.launch:
        conv.set_launch(*[int(x) for x in args.launch.split(",")])
    elif not args.no_tune:
        conv.autotune(dev, deep, shallow, reps=5)
    torch.cuda.synchronize()

    for _ in range(args.warmup):
        conv.step(dev, deep, shallow)
    torch.cuda.synchronize()
    print("[bench] warmup done", file=sys.stderr, flush=True)

    conv.timing_start(args.steps)
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    e0.record(stream)
    for _ in range(args.steps):
        conv.step(dev, deep, shallow)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    ms_step = e0.elapsed_time(e1) / args.steps
    kms, ncalls = conv.timing_read()
    conv.timing_start(0)
    kavg = {k: v / max(ncalls, 1) for k, v in kms.items()}

    # Per-step spread: the same number of steps again, an event pair around each.
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(args.steps)]
    for a, b in evs:
        a.record(stream)
        conv.step(dev, deep, shallow)
        b.record(stream)
    torch.cuda.synchronize()
    per_step = sorted(a.elapsed_time(b) for a, b in evs)
    copy_gbs = copy_bandwidth(torch)

    if args.calibrate_copy:
        nb = args.calibrate_copy * (1 << 20)
        src = torch.ones(nb // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    trig = deep["trig"].cpu().numpy()
    dst = deep["status"].cpu().numpy()
    sst = shallow["status"].cpu().numpy()
    kb = kernel_bytes(NLEV, n, trig, sst)
    dom = max(("trigger", "deep_plume", "shallow_retrigger"), key=lambda k: kavg[k])
    achieved = kb[dom] / (kavg[dom] * 1e-3) / 1e9
    step_bytes = bytes_per_column(NLEV)["total"] * n
    value = n / (ms_step * 1e-3)

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "columns/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "ms_per_step_median": per_step[len(per_step) // 2],
        "ms_per_step_min": per_step[0],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "conv_step (deep then shallow), 1152x768 = 884,736 columns x 30 "
                               "levels, latitude-clustered synthetic soundings, dt=1800 s",
                   "ncol": n, "nlev": NLEV},
        "roofline": {"bound": "hbm", "kernel": f"k_{dom}", "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": measured_traffic(f"k_{dom}"),
                     "algorithmic_bytes_per_launch": int(kb[dom]),
                     "avg_launch_ms": kavg[dom]},
        "step_roofline": {"algorithmic_bytes": int(step_bytes),
                          "bytes_per_column": bytes_per_column(NLEV)["total"],
                          "achieved_GBs": step_bytes / (ms_step * 1e-3) / 1e9,
                          "frac": step_bytes / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS,
                          "copy_GBs": copy_gbs,
                          "frac_of_copy": step_bytes / (ms_step * 1e-3) / 1e9 / copy_gbs},
        "kernels_ms": kavg,
        "launch_waves_per_cu": conv.get_launch(),
        "active_fraction": {"deep": float((dst == 0).mean()), "deep_triggered": float(trig.mean()),
                            "shallow": float((sst == 0).mean())},
        "wall_s_timed": wall,
    }

    if not args.no_extras:
        out["tracers"] = bench_tracers(torch, B, conv, dev, deep, shallow, max(args.steps, 10))
        print("[bench] tracers done", file=sys.stderr, flush=True)
        out["momentum"] = bench_momentum(torch, B, conv, dev, deep, shallow, max(args.steps, 10))
        print("[bench] momentum done", file=sys.stderr, flush=True)
        out["dilute"] = bench_dilute(torch, B, dev, n, max(args.steps, 10))
        print("[bench] dilute done", file=sys.stderr, flush=True)
        out["adjoint"] = bench_adjoint(torch, B, S, max(args.steps, 10))
        print("[bench] adjoint done", file=sys.stderr, flush=True)
        out["ensemble"] = bench_ensemble(torch, B, S, dev, deep, shallow, max(args.steps, 10),
                                         tune=not args.no_tune)
        print("[bench] ensemble done", file=sys.stderr, flush=True)
        if args.surrogate_n > 0:
            conv.step(dev, deep, shallow)  # the truth on the grid (the ensemble rewrote it)
            out["surrogate"] = bench_surrogate(torch, B, dev, deep, shallow, ms_step,
                                               args.surrogate_n, args.surrogate_epochs,
                                               max(args.steps, 10))
            print("[bench] surrogate done", file=sys.stderr, flush=True)

    if not args.no_cpu:
        threads = min(16, len(os.sched_getaffinity(0)))
        # The paper's own technique on the host: OpenMP dynamic scheduling, swept over the chunk
        # sizes of its Table "Effect of OpenMP dynamic chunk sizes" (Methodology); the best is
        # the baseline.
        sweep = {}
        for c in OMP_CHUNKS:
            rate, secs, nsteps = cpu_baseline(st, threads, chunk=c, min_cpu_s=8.0)
            sweep[c] = (rate, secs, nsteps)
            print(f"[bench] cpu oracle chunk {c}: {rate:.3e} columns/s", file=sys.stderr,
                  flush=True)
        best = max(sweep, key=lambda c: sweep[c][0])
        rate, secs, nsteps = sweep[best]
        out["cpu_baseline"] = {"value": rate, "unit": "columns/s", "cores": threads,
                               "kind": "oracle",
                               "sample": f"the full {n}-column grid, {nsteps} oracle steps "
                                         f"(OpenMP dynamic schedule, best chunk {best} of "
                                         f"{list(OMP_CHUNKS)}), {secs:.1f} s wall on {threads} "
                                         f"threads",
                               "cpu_model": cpu_model(), "nproc": os.cpu_count(),
                               "omp_chunk_sweep": {str(c): v[0] for c, v in sweep.items()}}
        ops, nsample = oracle_ops(st)
        out["cpu_baseline"]["oracle_ops_per_column"] = {
            "value": ops, "sample": f"every 16th column ({nsample} columns)",
            "rule": "+, -, *, /, sqrt, exp, log count 1 each (the oracle's own algorithm)"}
        out["step_roofline"]["ops_per_column"] = ops
        out["step_roofline"]["ops_per_byte"] = ops / bytes_per_column(NLEV)["total"]
        r1, s1, n1 = cpu_one_thread(st)
        out["cpu_baseline"]["one_thread"] = {
            "value": r1, "unit": "columns/s", "cores": 1,
            "sample": f"the full {n1}-column grid, one plain single-threaded oracle step, "
                      f"{s1:.1f} s"}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
