// mlp.hip -- the surrogate network's kernels for gfx950 (include/mlp.h): one tiled BF16 GEMM on
// the matrix cores (v_mfma_f32_32x32x16_bf16, FP32 accumulation) with fused epilogues, used for the
// forward layers (bias + GELU), the backward data gradient (times GELU') and, on batch-contiguous
// (transposed) copies with the batch split across blocks, the weight gradients; plus the bias
// gradients' row sums, MSE and Adam (which also refreshes the weights' BF16 copies).  In training
// the forward and data-gradient products write the transposed copies from their epilogues.
//
// GEMM tiling: a block computes a BM x BN tile (128 x 128, 256 x 256 or 128 x 64, chosen by shape)
// with its wavefronts in a WM x WN arrangement, each owning (BM/WM) x (BN/WN) as 32 x 32 MFMA
// tiles.  K advances 64 at a time through two LDS stages: the next K tile goes from global memory
// straight into the other stage (global_load_lds_dwordx4, no register staging) while the current
// one feeds the MFMAs; every row of a tile is one full 128-byte line, stored with its 16-byte
// chunks XOR-swizzled by the row pair so that fragment reads are free of bank conflicts.  Block ids are mapped so that the N tiles of one M tile run on the
// same XCD (the hardware deals consecutive blocks to the 8 XCDs in turn), so an activation tile is
// fetched into one XCD's L2 once and reused there; products with fewer M tiles than XCDs take
// their tiles in plain order.  The epilogue stages each wavefront's
// accumulators in LDS 32 rows at a time and finishes them in chunks of 8 consecutive columns of a
// row, so that bias, pre-activation and outputs move in 16-byte loads and stores; a transposed
// copy is gathered column by column from the same strips.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdint.h>
#include <string.h>

#include <atomic>
#include <vector>

#include "mlp.h"
#include "mlp_internal.hpp"

namespace {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16;
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

constexpr int THREADS = 256;  // block size of the elementwise and reduction kernels
constexpr int BK = 64;
constexpr int LDS_ROW = BK + 8;  // bf16 per row when sizing a block's LDS (the epilogue's strips
                                 // need more than the operand stages' unpadded rows)
constexpr int NXCD = 8;

thread_local int g_mlp_hip = 0;

__device__ __forceinline__ uint16_t f2bf(float f) {  // round to nearest even
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

using mlpk::gelu;
using mlpk::gelu_grad;

enum Mode : int {
    EPI_F32 = 0,      // c (float) = acc + bias
    EPI_GELU = 1,     // c (bf16) = gelu(acc + bias); z (float) = acc + bias
    EPI_DGELU = 2,    // c (bf16) = acc * gelu'(z)
    EPI_PARTIAL = 3,  // c (float) + blockIdx.y * split_stride = acc
};

struct GemmArgs {
    const uint16_t *a, *b;
    int64_t lda, ldb;
    int64_t M;
    int N, K;
    int tiles_m, tiles_n;
    int xmap;    // XCD-grouped block order (at least NXCD tiles along M), else row-major tiles
    int ksplit;  // > 0: blockIdx.y covers K range [y*ksplit, (y+1)*ksplit)
    int mode;
    int vec;     // 16-byte epilogue accesses allowed (alignment of c, z, bias, ldc, split_stride)
    const float *bias;
    void *c;
    int64_t ldc;
    float *z;  // EPI_GELU output / EPI_DGELU input, leading dimension ldc
    int64_t split_stride;
    // EPI_GELU / EPI_DGELU: optional transposed copy of the bf16 output, ct[n * ldt + m] for
    // m < ldt (rows M <= m < ldt are zero), so that a later product can read it along the batch.
    // Tiles with at most 64 columns per wavefront only; ldt % 8 == 0 and ct 16-byte aligned.
    uint16_t *ct;
    int64_t ldt;
    int nt;      // BF16 output not re-read soon (inference): non-temporal stores
};

template <int BM, int BN, int WM, int WN>
constexpr size_t gemm_lds_bytes() {
    return (size_t)2 * (BM + BN) * LDS_ROW * sizeof(uint16_t);
}

template <int BM, int BN, int WM, int WN>
__global__ __launch_bounds__(WM * WN * 64) void k_gemm(GemmArgs g) {
    constexpr int NT = WM * WN * 64;
    constexpr int TM = BM / WM / 32, TN = BN / WN / 32;  // 32 x 32 MFMA tiles per wavefront
    constexpr int SW = 32 * TN, SLD = SW + 4;  // epilogue strip: 32 rows x SW columns (floats)
    static_assert(WM * WN * 32 * SLD * sizeof(float) <= gemm_lds_bytes<BM, BN, WM, WN>(),
                  "epilogue strips must fit in the operand buffers");
    extern __shared__ __attribute__((aligned(16))) uint16_t smem[];

    const int t = threadIdx.x, lane = t & 63, w = t >> 6, wm = w / WN, wn = w % WN;
    const int64_t bid = blockIdx.x;
    int tn;
    int64_t tm;
    if (g.xmap) {
        const int xcd = (int)(bid % NXCD);
        const int64_t j = bid / NXCD;
        tn = (int)(j % g.tiles_n);
        tm = (j / g.tiles_n) * NXCD + xcd;
        if (tm >= g.tiles_m) return;
    } else {
        tn = (int)(bid % g.tiles_n);
        tm = bid / g.tiles_n;
    }
    const int64_t m0 = tm * BM;
    const int n0 = tn * BN;
    int k0 = 0, k1 = g.K;
    if (g.ksplit > 0) {
        k0 = blockIdx.y * g.ksplit;
        k1 = min(k0 + g.ksplit, g.K);
    }

    f32x16 acc[TM][TN];
#pragma unroll
    for (int a = 0; a < TM; ++a)
#pragma unroll
        for (int b = 0; b < TN; ++b)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[a][b][r] = 0.0f;

    // Operand tiles in LDS without padding: row r of a stage is 64 BF16 (128 bytes, eight 16-byte
    // chunks) and its k-chunk c sits at chunk position c ^ ((r >> 1) & 7).  With 64 four-byte
    // banks, two 128-byte rows share one bank cycle; the swizzle gives the 16 consecutive rows that
    // a fragment read serves together 16 distinct 16-byte bank groups.  Whole K tiles go global ->
    // LDS directly (one 16-byte chunk per lane, eight rows per wavefront instruction: lane i fills
    // position i & 7 of row i >> 3 and so fetches the chunk that belongs there); rows past M or N
    // read row M-1 or N-1 instead (their results are discarded).  A tile cut by the K limit goes
    // through registers with zero fill.
    constexpr int SROW = BK;                      // bf16 per LDS row
    constexpr int STAGE_A = BM * SROW, STAGE_B = BN * SROW;
    auto SA = [&](int buf) { return smem + buf * STAGE_A; };
    auto SB = [&](int buf) { return smem + 2 * STAGE_A + buf * STAGE_B; };
    constexpr int NWV = WM * WN;
    static_assert(BM % (8 * NWV) == 0 && BN % (8 * NWV) == 0, "rows per wavefront instruction");
    auto stage_direct = [&](const uint16_t *p, int64_t ld, int64_t r0, int64_t rlim, int kk,
                            uint16_t *dst, int rows) {
        const int lr = lane >> 3, pos = lane & 7;
        for (int j = 0; j < rows / (8 * NWV); ++j) {
            const int R0 = (j * NWV + w) * 8;
            int64_t r = r0 + R0 + lr;
            r = r < rlim ? r : rlim - 1;
            const uint16_t *src = p + r * ld + kk + 8 * (pos ^ (((R0 + lr) >> 1) & 7));
            __builtin_amdgcn_global_load_lds((__attribute__((address_space(1))) void *)src,
                                             (__attribute__((address_space(3))) void *)(dst + R0 * SROW),
                                             16, 0, 0);
        }
    };
    auto stage_regs = [&](const uint16_t *p, int64_t ld, int64_t r0, int64_t rlim, int kk, int klim,
                          uint16_t *dst, int rows) {
        for (int idx = t; idx < rows * 8; idx += NT) {
            const int rr = idx >> 3, c = idx & 7;
            const int64_t r = r0 + rr;
            const int k = kk + 8 * c;
            uint4 v = make_uint4(0u, 0u, 0u, 0u);
            if (r < rlim && k < klim) v = *(const uint4 *)(p + r * ld + k);
            *(uint4 *)(dst + rr * SROW + 8 * (c ^ ((rr >> 1) & 7))) = v;
        }
    };
    auto stage = [&](int buf, int kk) {
        if (kk + BK <= k1) {
            stage_direct(g.a, g.lda, m0, g.M, kk, SA(buf), BM);
            stage_direct(g.b, g.ldb, n0, g.N, kk, SB(buf), BN);
        } else {
            stage_regs(g.a, g.lda, m0, g.M, kk, k1, SA(buf), BM);
            stage_regs(g.b, g.ldb, n0, g.N, kk, k1, SB(buf), BN);
        }
    };

    const int nk = k1 > k0 ? (k1 - k0 + BK - 1) / BK : 0;
    if (nk > 0) stage(0, k0);
    __builtin_amdgcn_s_waitcnt(0x0f70);  // vmcnt(0): the direct loads have landed
    __syncthreads();
    const int lrow = lane & 31, lk = 8 * (lane >> 5);
    for (int kt = 0; kt < nk; ++kt) {
        const int cur = kt & 1;
        if (kt + 1 < nk) stage(cur ^ 1, k0 + (kt + 1) * BK);
        const uint16_t *Ac = SA(cur), *Bc = SB(cur);
#pragma unroll
        for (int ks = 0; ks < BK; ks += 16) {
            const int c = (ks + lk) >> 3;
            bf16x8 af[TM], bf[TN];
#pragma unroll
            for (int a = 0; a < TM; ++a) {
                const int r = wm * (BM / WM) + a * 32 + lrow;
                af[a] = *(const bf16x8 *)&Ac[r * SROW + 8 * (c ^ ((r >> 1) & 7))];
            }
#pragma unroll
            for (int b = 0; b < TN; ++b) {
                const int r = wn * (BN / WN) + b * 32 + lrow;
                bf[b] = *(const bf16x8 *)&Bc[r * SROW + 8 * (c ^ ((r >> 1) & 7))];
            }
#pragma unroll
            for (int a = 0; a < TM; ++a)
#pragma unroll
                for (int b = 0; b < TN; ++b)
                    acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(af[a], bf[b], acc[a][b], 0, 0, 0);
        }
        __builtin_amdgcn_s_waitcnt(0x0f70);  // vmcnt(0): the next stage has landed
        __syncthreads();
    }

    // Epilogue.  Accumulator layout of a 32x32 MFMA tile: register r of lane l holds row
    // 8*(r/4) + 4*(l/32) + r%4, column l%32.  Each wavefront writes one 32-row strip of its tile to
    // its own LDS region, then each lane finishes chunks of 8 consecutive columns of one row.
    float *strip = (float *)smem + w * 32 * SLD;
    constexpr int CPR = SW / 8;          // chunks per strip row
    constexpr int NCH = 32 * CPR / 64;   // chunks per lane per strip
    static_assert((32 * CPR) % 64 == 0, "strip chunks must divide among the lanes");
    const bool use_bias = g.bias && (g.mode == EPI_F32 || g.mode == EPI_GELU);
    // Transposed copy: lane c of the wavefront owns column c of its strips and gathers the
    // finished values of its TM * 32 rows, two BF16 per register.
    constexpr bool CT_OK = SW <= 64;
    constexpr int TLD = TM * 32 + 8;  // row stride (bf16) of the transposed tile T in LDS
    static_assert(!CT_OK || WM * WN * (32 * SLD * sizeof(float) + SW * TLD * sizeof(uint16_t)) <=
                                gemm_lds_bytes<BM, BN, WM, WN>(),
                  "strips and transposed tiles must fit in the operand buffers");
    const bool ct = CT_OK && g.ct != nullptr;
    const int64_t mw = m0 + wm * (BM / WM);  // first row of this wavefront
    uint32_t pk[CT_OK ? TM * 16 : 1];
#pragma unroll
    for (int a = 0; a < TM; ++a) {
#pragma unroll
        for (int b = 0; b < TN; ++b)
#pragma unroll
            for (int r = 0; r < 16; ++r)
                strip[(8 * (r >> 2) + 4 * (lane >> 5) + (r & 3)) * SLD + b * 32 + lrow] = acc[a][b][r];
        __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0): the strip is written
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int i = 0; i < NCH; ++i) {
            const int ch = lane + i * 64;
            const int rr = ch / CPR, cc = (ch % CPR) * 8;
            const int64_t m = m0 + wm * (BM / WM) + a * 32 + rr;
            const int n = n0 + wn * (BN / WN) + cc;
            if (m >= g.M || n >= g.N) continue;
            const int cnt = min(8, g.N - n);
            const bool full = g.vec && cnt == 8;
            float v[8], x[8];
            *(float4 *)&v[0] = *(const float4 *)&strip[rr * SLD + cc];
            *(float4 *)&v[4] = *(const float4 *)&strip[rr * SLD + cc + 4];
            if (use_bias) {
                if (full) {
                    *(float4 *)&x[0] = *(const float4 *)&g.bias[n];
                    *(float4 *)&x[4] = *(const float4 *)&g.bias[n + 4];
                } else {
#pragma unroll
                    for (int e = 0; e < 8; ++e) x[e] = e < cnt ? g.bias[n + e] : 0.0f;
                }
#pragma unroll
                for (int e = 0; e < 8; ++e) v[e] += x[e];
            }
            const int64_t o = m * g.ldc + n;
            if (g.mode == EPI_F32 || g.mode == EPI_PARTIAL) {
                float *c = (float *)g.c + o;
                if (g.mode == EPI_PARTIAL) c += (int64_t)blockIdx.y * g.split_stride;
                if (full) {
                    *(float4 *)&c[0] = *(float4 *)&v[0];
                    *(float4 *)&c[4] = *(float4 *)&v[4];
                } else {
#pragma unroll
                    for (int e = 0; e < 8; ++e)
                        if (e < cnt) c[e] = v[e];
                }
                continue;
            }
            if (g.mode == EPI_GELU) {
                if (g.z) {
                    if (full) {
                        *(float4 *)&g.z[o] = *(float4 *)&v[0];
                        *(float4 *)&g.z[o + 4] = *(float4 *)&v[4];
                    } else {
#pragma unroll
                        for (int e = 0; e < 8; ++e)
                            if (e < cnt) g.z[o + e] = v[e];
                    }
                }
#pragma unroll
                for (int e = 0; e < 8; ++e) v[e] = gelu(v[e]);
            } else {  // EPI_DGELU
                if (full) {
                    *(float4 *)&x[0] = *(const float4 *)&g.z[o];
                    *(float4 *)&x[4] = *(const float4 *)&g.z[o + 4];
                } else {
#pragma unroll
                    for (int e = 0; e < 8; ++e) x[e] = e < cnt ? g.z[o + e] : 0.0f;
                }
#pragma unroll
                for (int e = 0; e < 8; ++e) v[e] *= gelu_grad(x[e]);
            }
            if (ct) {  // the finished values back into the strip for the column gather
                *(float4 *)&strip[rr * SLD + cc] = *(float4 *)&v[0];
                *(float4 *)&strip[rr * SLD + cc + 4] = *(float4 *)&v[4];
            }
            uint16_t *c = (uint16_t *)g.c + o;
            if (full) {
                uint32_t h[4];
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    h[e] = mlpk::bf16x2(v[2 * e], v[2 * e + 1]);
                if (g.nt) {
                    const u32x4 hv = {h[0], h[1], h[2], h[3]};
                    __builtin_nontemporal_store(hv, (u32x4 *)c);
                } else {
                    *(uint4 *)c = make_uint4(h[0], h[1], h[2], h[3]);
                }
            } else {
#pragma unroll
                for (int e = 0; e < 8; ++e)
                    if (e < cnt) c[e] = f2bf(v[e]);
            }
        }
        if constexpr (CT_OK) {
            if (ct) {
                __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0): finished values are in the strip
                __builtin_amdgcn_wave_barrier();
                if (lane < SW) {
#pragma unroll
                    for (int rr = 0; rr < 32; rr += 2) {
                        const int64_t m = mw + a * 32 + rr;
                        pk[a * 16 + rr / 2] =
                            mlpk::bf16x2(m < g.M ? strip[rr * SLD + lane] : 0.0f,
                                         m + 1 < g.M ? strip[(rr + 1) * SLD + lane] : 0.0f);
                    }
                }
            }
        }
        __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0): the strip is read before it is reused
        __builtin_amdgcn_wave_barrier();
    }
    if constexpr (CT_OK) {
        // Through LDS once more so that each store instruction covers whole lines: lane c puts its
        // column (TM * 32 rows, 16 bytes per 8 rows) in row c of T, then the wavefront stores
        // 64 / PIECES columns per instruction, PIECES lanes per column.
        constexpr int PIECES = TM * 4, CPI = 64 / PIECES;
        static_assert(64 % PIECES == 0 && SW % CPI == 0, "column pieces must tile the wavefront");
        if (ct) {
            uint16_t *T = (uint16_t *)((float *)smem + WM * WN * 32 * SLD) + w * SW * TLD;
            if (lane < SW) {
#pragma unroll
                for (int q = 0; q < PIECES; ++q)
                    *(uint4 *)&T[lane * TLD + 8 * q] =
                        make_uint4(pk[4 * q], pk[4 * q + 1], pk[4 * q + 2], pk[4 * q + 3]);
            }
            __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0): T is written
            __builtin_amdgcn_wave_barrier();
            const int piece = lane % PIECES;
            const int64_t m = mw + 8 * piece;  // ldt % 8 == 0: a piece below ldt is whole
#pragma unroll
            for (int i = 0; i < SW / CPI; ++i) {
                const int col = i * CPI + lane / PIECES;
                const int n = n0 + wn * (BN / WN) + col;
                if (n < g.N && m < g.ldt)
                    *(uint4 *)(g.ct + (int64_t)n * g.ldt + m) =
                        *(const uint4 *)&T[col * TLD + 8 * piece];
            }
        }
    }
}

template <int BM, int BN, int WM, int WN>
int launch_tiles(GemmArgs g, int splits, hipStream_t st) {
    g.tiles_m = (int)((g.M + BM - 1) / BM);
    g.tiles_n = (g.N + BN - 1) / BN;
    // With fewer M tiles than XCDs (the weight gradients' few tiles, split along K), grouping by
    // XCD would leave XCDs idle: tiles then go in plain order and the splits spread them.
    g.xmap = g.tiles_m >= NXCD;
    const int64_t mgroups = (g.tiles_m + NXCD - 1) / NXCD;
    const int64_t blocks = g.xmap ? mgroups * NXCD * g.tiles_n : (int64_t)g.tiles_m * g.tiles_n;
    if (blocks <= 0 || blocks > 0x7fffffff || splits < 1) return MLP_EINVAL;
    constexpr size_t lds = gemm_lds_bytes<BM, BN, WM, WN>();
    // The LDS limit above 64 KiB is a per-device function attribute: set once per device.
    static std::atomic<uint64_t> done{0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return MLP_EHIP;
    if (!(done.load() & (1ull << dev))) {
        if (hipFuncSetAttribute((const void *)k_gemm<BM, BN, WM, WN>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
            return MLP_EHIP;
        done.fetch_or(1ull << dev);
    }
    hipLaunchKernelGGL((k_gemm<BM, BN, WM, WN>), dim3((unsigned)blocks, (unsigned)splits),
                       dim3(WM * WN * 64), lds, st, g);
    return MLP_OK;
}

bool al16(const void *p) { return ((uintptr_t)p & 15u) == 0; }

// Tile shape by problem shape: 128 x 64 for narrow outputs, 256 x 256 when the grid still has
// several blocks per compute unit, else 128 x 128.
int launch_gemm(const GemmArgs &in, int splits, hipStream_t st) {
    GemmArgs g = in;
    g.vec = al16(g.c) && (!g.z || al16(g.z)) && (!g.bias || al16(g.bias)) && g.ldc % 8 == 0 &&
            g.split_stride % 8 == 0;
    if (g.ct) {  // the transposed copy needs at most 64 columns per wavefront
        if (!al16(g.ct) || g.ldt % 8 != 0 || g.ldt < g.M || (g.mode != EPI_GELU && g.mode != EPI_DGELU))
            return MLP_EINVAL;
        if (g.N <= 64) return launch_tiles<128, 64, 2, 2>(g, splits, st);
        return launch_tiles<128, 128, 2, 2>(g, splits, st);
    }
    if (g.N <= 64) return launch_tiles<128, 64, 2, 2>(g, splits, st);
    const int64_t big = ((g.M + 255) / 256) * ((g.N + 255) / 256) * splits;
    if (g.N % 256 == 0 && big >= 1024) return launch_tiles<256, 256, 4, 2>(g, splits, st);
    return launch_tiles<128, 128, 2, 2>(g, splits, st);
}

// out[c][r] = in[r][c] for r < rows, c < cols; out[c][r] = 0 for rows <= r < ldo (row padding).
// 64 x 64 tiles through LDS so that both sides are read and written along rows.
constexpr int TT = 64;
__global__ __launch_bounds__(THREADS) void k_transpose(const uint16_t *in, int64_t rows, int cols,
                                                       int64_t ldo, uint16_t *out) {
    __shared__ uint16_t sh[TT][TT + 2];
    const int c0 = blockIdx.x * TT;
    const int64_t r0 = (int64_t)blockIdx.y * TT;
    const int j = threadIdx.x % TT, i0 = threadIdx.x / TT;
    for (int i = i0; i < TT; i += THREADS / TT) {
        const int64_t r = r0 + i;
        const int c = c0 + j;
        sh[i][j] = (r < rows && c < cols) ? in[r * cols + c] : (uint16_t)0;
    }
    __syncthreads();
    for (int i = i0; i < TT; i += THREADS / TT) {
        const int c = c0 + i;
        const int64_t r = r0 + j;
        if (c < cols && r < ldo) out[(int64_t)c * ldo + r] = sh[j][i];
    }
}

// ------------------------------------------------------------------ reductions, loss, optimiser
// out[r] = sum over b < ld of x[r*ld + b] (bf16; ld % 8 == 0, the padding past the batch is zero):
// one block per row, 16-byte loads, each thread's values summed in a fixed order, then a
// fixed-shape tree.
__global__ __launch_bounds__(THREADS) void k_rowsum(const uint16_t *x, int64_t ld, float *out) {
    __shared__ float sh[THREADS];
    const uint16_t *row = x + (int64_t)blockIdx.x * ld;
    float s[2] = {0.0f, 0.0f};
    for (int64_t b = (int64_t)threadIdx.x * 8; b < ld; b += THREADS * 8) {
        const uint4 v = *(const uint4 *)(row + b);
        const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            s[0] += __uint_as_float(w[e] << 16);
            s[1] += __uint_as_float(w[e] & 0xFFFF0000u);
        }
    }
    sh[threadIdx.x] = s[0] + s[1];
    __syncthreads();
    for (int h = THREADS / 2; h > 0; h /= 2) {
        if ((int)threadIdx.x < h) sh[threadIdx.x] += sh[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[blockIdx.x] = sh[0];
}

// out[i] = sum over s < S of part[s*len + i]: a block takes 64 consecutive outputs, wavefront g
// of its four sums partials g, g + 4, g + 8, ... in order, and the four sums are added in a fixed
// order (so each output has four independent load chains instead of one).
constexpr int SUM_COLS = 64;
static_assert(THREADS == 4 * SUM_COLS, "k_sum_parts adds four wavefronts' sums");
__global__ __launch_bounds__(THREADS) void k_sum_parts(const float *part, int S, int64_t len,
                                                       float *out) {
    __shared__ float sh[THREADS];
    const int o = threadIdx.x % SUM_COLS, g = threadIdx.x / SUM_COLS;
    const int64_t i = (int64_t)blockIdx.x * SUM_COLS + o;
    float s = 0.0f;
    if (i < len) {
#pragma unroll 4
        for (int k = g; k < S; k += THREADS / SUM_COLS) s += part[(int64_t)k * len + i];
    }
    sh[threadIdx.x] = s;
    __syncthreads();
    if (g == 0 && i < len)
        out[i] = (sh[o] + sh[SUM_COLS + o]) + (sh[2 * SUM_COLS + o] + sh[3 * SUM_COLS + o]);
}

__device__ float block_sum(float v) {  // fixed-shape tree over the block; result in thread 0
    __shared__ float sh[THREADS];
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int h = THREADS / 2; h > 0; h /= 2) {
        if ((int)threadIdx.x < h) sh[threadIdx.x] += sh[threadIdx.x + h];
        __syncthreads();
    }
    return sh[0];
}

// Per element of y[batch][w]: d = y - t; dz = bf16(scale * 2 d) for j < nv, else 0; block partial
// sums of d^2 over j < nv.
__global__ __launch_bounds__(THREADS) void k_mse(const float *y, const float *t, int64_t total, int w,
                                                 int nv, float scale, uint16_t *dz, float *part) {
    const int64_t i = (int64_t)blockIdx.x * THREADS + threadIdx.x;
    float sq = 0.0f;
    if (i < total) {
        const int jj = (int)(i % w);
        const float d = y[i] - t[i];
        const bool ok = jj < nv;
        dz[i] = ok ? f2bf(2.0f * d * scale) : (uint16_t)0;
        sq = ok ? d * d : 0.0f;
    }
    const float s = block_sum(sq);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ __launch_bounds__(THREADS) void k_mse_final(const float *part, int64_t n, float scale,
                                                       float *loss) {
    float s = 0.0f;
    for (int64_t i = threadIdx.x; i < n; i += THREADS) s += part[i];
    const float tot = block_sum(s);
    if (threadIdx.x == 0) loss[0] = tot * scale;
}

// Where each layer's weights sit in the parameter vector, and their BF16 copies.
struct BfMap {
    int n;
    int64_t poff[MLP_MAX_LAYERS];
    int no[MLP_MAX_LAYERS], ni[MLP_MAX_LAYERS];
    uint16_t *wb[MLP_MAX_LAYERS], *wt[MLP_MAX_LAYERS];
};

// Adam on every parameter; a weight's new value also goes to its BF16 copies: wb (the layout of
// W [no][ni]) and wt (transposed, [ni][no]).
__global__ __launch_bounds__(THREADS) void k_adam(float *p, const float *g, float *m, float *v,
                                                  int64_t n, float lr, float b1, float b2, float eps,
                                                  float bc1, float bc2, BfMap bm) {
    const int64_t i = (int64_t)blockIdx.x * THREADS + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float pi = p[i] - lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
    p[i] = pi;
    int64_t off = i;
    int no = 0, ni = 0;
    uint16_t *wb = nullptr, *wt = nullptr;
#pragma unroll
    for (int l = 0; l < MLP_MAX_LAYERS; ++l)  // the layer holding parameter i
        if (l < bm.n && i >= bm.poff[l]) {
            off = i - bm.poff[l];
            no = bm.no[l];
            ni = bm.ni[l];
            wb = bm.wb[l];
            wt = bm.wt[l];
        }
    if (off < (int64_t)no * ni) {  // a weight, not a bias
        const uint16_t h = f2bf(pi);
        const int r = (int)(off / ni), c = (int)(off % ni);
        wb[off] = h;
        wt[(int64_t)c * no + r] = h;
    }
}

// BF16 copies of W [rows][cols]: wb (same layout) and wt (transposed [cols][rows]).
__global__ __launch_bounds__(THREADS) void k_to_bf16(const float *W, int rows, int cols, uint16_t *wb,
                                                     uint16_t *wt) {
    const int64_t i = (int64_t)blockIdx.x * THREADS + threadIdx.x;
    if (i >= (int64_t)rows * cols) return;
    const int r = (int)(i / cols), c = (int)(i % cols);
    const uint16_t h = f2bf(W[i]);
    wb[i] = h;
    wt[(int64_t)c * rows + r] = h;
}

__global__ __launch_bounds__(THREADS) void k_fill0(float *p, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * THREADS + threadIdx.x;
    if (i < n) p[i] = 0.0f;
}

unsigned nblocks(int64_t n) { return (unsigned)((n + THREADS - 1) / THREADS); }
size_t al256(size_t x) { return (x + 255) & ~size_t(255); }

int check() {
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        g_mlp_hip = (int)e;
        return MLP_EHIP;
    }
    return MLP_OK;
}

// Weight-gradient GEMM split: enough blocks to fill the chip, chunks a multiple of BK.
void wgrad_split(int64_t batch, int M, int N, int *S, int *chunk) {
    const int tiles = ((M + 127) / 128) * (N <= 64 ? 1 : (N + 127) / 128);
    int s = (512 + tiles - 1) / tiles;
    if (s > 64) s = 64;
    if (s < 1) s = 1;
    int64_t c = (batch + s - 1) / s;
    c = (c + BK - 1) / BK * BK;
    if (c < BK) c = BK;
    *chunk = (int)c;
    *S = (int)((batch + c - 1) / c);
    if (*S < 1) *S = 1;
}

constexpr int MAX_SPLIT = 64;

struct Layout {
    size_t params, grads, am, av, wb[MLP_MAX_LAYERS], wt[MLP_MAX_LAYERS];
    size_t act[MLP_MAX_LAYERS], zf[MLP_MAX_LAYERS], dz[2], part, lpart, total;
    // Batch-contiguous (transposed) copies for the weight gradients, rows of ldt = max_batch
    // rounded up to 8: actT[i] [w_i][ldt] written by the forward with keep, dzT [w][ldt] the
    // current layer's output gradient, xT [w_0][ldt] the input.
    size_t actT[MLP_MAX_LAYERS], dzT, xT;
    int64_t P;
    int64_t poff[MLP_MAX_LAYERS];  // offset of W_l in the parameter vector (b_l follows)
};

bool widths_ok(const int32_t *w, int n) {
    if (!w || n < 1 || n > MLP_MAX_LAYERS) return false;
    for (int i = 0; i <= n; ++i)
        if (w[i] < 32 || w[i] > 4096 || w[i] % 32 != 0) return false;
    return true;
}

// maxb: rows of an inference forward and of mlp_mse; maxt (<= maxb): rows of a training forward
// (keep) and backward, the only users of the pre-activations, the transposed copies and the hidden
// gradients.
Layout make_layout(const int32_t *w, int n, int64_t maxb, int64_t maxt) {
    Layout l{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = al256(off + bytes);
        return o;
    };
    int64_t P = 0;
    int wmax = 0;
    size_t pmax = 0;
    for (int i = 0; i < n; ++i) {
        l.poff[i] = P;
        P += (int64_t)w[i + 1] * w[i] + w[i + 1];
        size_t need = (size_t)MAX_SPLIT * w[i + 1] * w[i];
        if (need > pmax) pmax = need;
    }
    for (int i = 0; i <= n; ++i) wmax = w[i] > wmax ? w[i] : wmax;
    l.P = P;
    l.params = take(P * sizeof(float));
    l.grads = take(P * sizeof(float));
    l.am = take(P * sizeof(float));
    l.av = take(P * sizeof(float));
    for (int i = 0; i < n; ++i) {
        l.wb[i] = take((size_t)w[i + 1] * w[i] * 2);
        l.wt[i] = take((size_t)w[i + 1] * w[i] * 2);
    }
    const size_t ldt = (size_t)(maxt + 7) / 8 * 8;
    for (int i = 1; i < n; ++i) {
        l.act[i] = take((size_t)maxb * w[i] * 2);
        l.zf[i] = take((size_t)maxt * w[i] * 4);
        l.actT[i] = take(ldt * w[i] * 2);
    }
    // dz[0]: the output gradient of mlp_mse (any batch) and a hidden gradient of mlp_backward
    const size_t dz0 = (size_t)maxb * w[n] > (size_t)maxt * wmax ? (size_t)maxb * w[n]
                                                                   : (size_t)maxt * wmax;
    l.dz[0] = take(dz0 * 2);
    l.dz[1] = take((size_t)maxt * wmax * 2);
    l.dzT = take(ldt * wmax * 2);
    l.xT = take(ldt * w[0] * 2);
    l.part = take(pmax * sizeof(float));
    l.lpart = take(((size_t)maxb * w[n] + THREADS - 1) / THREADS * sizeof(float));
    l.total = off;
    return l;
}

}  // namespace

struct mlp {
    int n;
    int32_t w[MLP_MAX_LAYERS + 1];
    int64_t maxb;
    int64_t maxt;          // rows of a training forward / backward (<= maxb)
    char *ws;
    Layout lay;
    int64_t t;             // Adam steps taken
    const uint16_t *x;     // input of the last forward with keep
    int64_t fwd_batch;
    int dz_top;            // buffer holding the output gradient of the last mlp_mse
};

namespace {

float *fp(mlp *m, size_t off) { return (float *)(m->ws + off); }
uint16_t *hp(mlp *m, size_t off) { return (uint16_t *)(m->ws + off); }

int refresh_bf16(mlp *m, hipStream_t st) {
    for (int i = 0; i < m->n; ++i) {
        const int64_t cnt = (int64_t)m->w[i + 1] * m->w[i];
        hipLaunchKernelGGL(k_to_bf16, dim3(nblocks(cnt)), dim3(THREADS), 0, st,
                           (const float *)fp(m, m->lay.params) + m->lay.poff[i], m->w[i + 1], m->w[i],
                           hp(m, m->lay.wb[i]), hp(m, m->lay.wt[i]));
    }
    return check();
}

}  // namespace

namespace mlpk {

NetView net_view(const mlp_t *mc) {
    mlp *m = const_cast<mlp *>(mc);
    NetView v{};
    v.n = m->n;
    for (int i = 0; i <= m->n; ++i) v.w[i] = m->w[i];
    for (int i = 0; i < m->n; ++i) {
        v.wb[i] = hp(m, m->lay.wb[i]);
        v.bias[i] = fp(m, m->lay.params) + m->lay.poff[i] + (int64_t)m->w[i + 1] * m->w[i];
    }
    return v;
}

}  // namespace mlpk

extern "C" {

size_t mlp_workspace_bytes_ex(const int32_t *widths, int n_layers, int64_t max_batch,
                              int64_t max_train_batch) {
    if (!widths_ok(widths, n_layers) || max_batch < 1 || max_batch > (1ll << 26) ||
        max_train_batch < 1 || max_train_batch > max_batch)
        return 0;
    return make_layout(widths, n_layers, max_batch, max_train_batch).total;
}

size_t mlp_workspace_bytes(const int32_t *widths, int n_layers, int64_t max_batch) {
    return mlp_workspace_bytes_ex(widths, n_layers, max_batch, max_batch);
}

int mlp_create_ex(const int32_t *widths, int n_layers, int64_t max_batch, int64_t max_train_batch,
                  void *workspace, size_t ws_bytes, mlp_t **out) {
    if (!out || !workspace || !widths_ok(widths, n_layers) || max_batch < 1 ||
        max_batch > (1ll << 26) || max_train_batch < 1 || max_train_batch > max_batch)
        return MLP_EINVAL;
    if (((uintptr_t)workspace & 255u) != 0) return MLP_EINVAL;
    const Layout l = make_layout(widths, n_layers, max_batch, max_train_batch);
    if (ws_bytes < l.total) return MLP_EINVAL;
    mlp *m = new mlp;
    m->n = n_layers;
    for (int i = 0; i <= n_layers; ++i) m->w[i] = widths[i];
    m->maxb = max_batch;
    m->maxt = max_train_batch;
    m->ws = (char *)workspace;
    m->lay = l;
    m->t = 0;
    m->x = nullptr;
    m->fwd_batch = 0;
    m->dz_top = 0;
    *out = m;
    return MLP_OK;
}

int mlp_create(const int32_t *widths, int n_layers, int64_t max_batch, void *workspace,
               size_t ws_bytes, mlp_t **out) {
    return mlp_create_ex(widths, n_layers, max_batch, max_batch, workspace, ws_bytes, out);
}

void mlp_destroy(mlp_t *m) { delete m; }

int64_t mlp_param_count(const mlp_t *m) { return m ? m->lay.P : -1; }

int mlp_set_params(mlp_t *m, const float *params, void *stream) {
    if (!m || !params) return MLP_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    const int64_t P = m->lay.P;
    if (hipMemcpyAsync(fp(m, m->lay.params), params, P * sizeof(float), hipMemcpyDeviceToDevice, st) !=
        hipSuccess) {
        g_mlp_hip = (int)hipGetLastError();
        return MLP_EHIP;
    }
    hipLaunchKernelGGL(k_fill0, dim3(nblocks(P)), dim3(THREADS), 0, st, fp(m, m->lay.am), P);
    hipLaunchKernelGGL(k_fill0, dim3(nblocks(P)), dim3(THREADS), 0, st, fp(m, m->lay.av), P);
    hipLaunchKernelGGL(k_fill0, dim3(nblocks(P)), dim3(THREADS), 0, st, fp(m, m->lay.grads), P);
    m->t = 0;
    return refresh_bf16(m, st);
}

int mlp_get_params(const mlp_t *m, float *params, void *stream) {
    if (!m || !params) return MLP_EINVAL;
    if (hipMemcpyAsync(params, m->ws + m->lay.params, m->lay.P * sizeof(float),
                       hipMemcpyDeviceToDevice, (hipStream_t)stream) != hipSuccess)
        return MLP_EHIP;
    return MLP_OK;
}

int mlp_get_grads(const mlp_t *m, float *grads, void *stream) {
    if (!m || !grads) return MLP_EINVAL;
    if (hipMemcpyAsync(grads, m->ws + m->lay.grads, m->lay.P * sizeof(float),
                       hipMemcpyDeviceToDevice, (hipStream_t)stream) != hipSuccess)
        return MLP_EHIP;
    return MLP_OK;
}

int mlp_forward(mlp_t *m, const uint16_t *x, float *y, int64_t batch, int keep, void *stream) {
    if (!m || !x || !y || batch < 1 || batch > (keep ? m->maxt : m->maxb)) return MLP_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    const uint16_t *in = x;
    for (int i = 0; i < m->n; ++i) {
        GemmArgs g{};
        g.a = in;
        g.lda = m->w[i];
        g.b = hp(m, m->lay.wb[i]);
        g.ldb = m->w[i];
        g.M = batch;
        g.N = m->w[i + 1];
        g.K = m->w[i];
        g.bias = fp(m, m->lay.params) + m->lay.poff[i] + (int64_t)m->w[i + 1] * m->w[i];
        if (i + 1 < m->n) {
            g.mode = EPI_GELU;
            g.c = hp(m, m->lay.act[i + 1]);
            if (keep) {
                g.z = fp(m, m->lay.zf[i + 1]);
                g.ct = hp(m, m->lay.actT[i + 1]);
                g.ldt = (batch + 7) / 8 * 8;
            } else {
                // inference: the activation is read once, by the next layer (3.94 -> 3.80 ms for
                // the surrogate on the 884,736-column grid); training keeps its outputs cached
                g.nt = 1;
            }
        } else {
            g.mode = EPI_F32;
            g.c = y;
        }
        g.ldc = m->w[i + 1];
        const int rc = launch_gemm(g, 1, st);
        if (rc != MLP_OK) return rc;
        in = (const uint16_t *)g.c;
    }
    if (keep) {
        m->x = x;
        m->fwd_batch = batch;
    }
    return check();
}

int mlp_mse(mlp_t *m, const float *y, const float *target, int64_t batch, int n_valid, float *loss,
            void *stream) {
    if (!m || !y || !target || !loss || batch < 1 || batch > m->maxb || n_valid < 1 ||
        n_valid > m->w[m->n])
        return MLP_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    const int wo = m->w[m->n];
    const int64_t total = batch * wo;
    const unsigned nb = nblocks(total);
    const float scale = (float)(1.0 / ((double)batch * n_valid));
    hipLaunchKernelGGL(k_mse, dim3(nb), dim3(THREADS), 0, st, y, target, total, wo, n_valid, scale,
                       hp(m, m->lay.dz[0]), fp(m, m->lay.lpart));
    hipLaunchKernelGGL(k_mse_final, dim3(1), dim3(THREADS), 0, st, (const float *)fp(m, m->lay.lpart),
                       (int64_t)nb, scale, loss);
    m->dz_top = 0;
    return check();
}

int mlp_backward(mlp_t *m, int64_t batch, void *stream) {
    if (!m || !m->x || batch != m->fwd_batch) return MLP_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    int cur = m->dz_top;
    float *part = fp(m, m->lay.part);
    // Weight gradients dW_i[no][ni] = sum_b dz[b][no] ain[b][ni] read both factors along the batch:
    // rows of ldt (the batch rounded up to 8, zero past it).  The hidden activations' copies come
    // from the forward, the hidden gradients' from the data-gradient products; the input's and
    // the output gradient's are transposed here.
    const int64_t ldt = (batch + 7) / 8 * 8;
    uint16_t *dzT = hp(m, m->lay.dzT), *xT = hp(m, m->lay.xT);
    const int wo = m->w[m->n], w0 = m->w[0];
    hipLaunchKernelGGL(k_transpose, dim3((wo + TT - 1) / TT, (unsigned)((ldt + TT - 1) / TT)),
                       dim3(THREADS), 0, st, (const uint16_t *)hp(m, m->lay.dz[cur]), batch, wo,
                       ldt, dzT);
    hipLaunchKernelGGL(k_transpose, dim3((w0 + TT - 1) / TT, (unsigned)((ldt + TT - 1) / TT)),
                       dim3(THREADS), 0, st, m->x, batch, w0, ldt, xT);
    for (int i = m->n - 1; i >= 0; --i) {
        const int no = m->w[i + 1], ni = m->w[i];
        const uint16_t *dz = hp(m, m->lay.dz[cur]);
        const uint16_t *aT = i == 0 ? xT : hp(m, m->lay.actT[i]);
        float *gW = fp(m, m->lay.grads) + m->lay.poff[i];
        float *gb = gW + (int64_t)no * ni;
        // dW: the NT kernel over the batch, split across blocks, partials summed in order.
        int S, chunk;
        wgrad_split(ldt, no, ni, &S, &chunk);
        GemmArgs g{};
        g.a = dzT;
        g.lda = ldt;
        g.b = aT;
        g.ldb = ldt;
        g.M = no;
        g.N = ni;
        g.K = (int)ldt;
        g.ksplit = chunk;
        g.mode = EPI_PARTIAL;
        g.c = part;
        g.ldc = ni;
        g.split_stride = (int64_t)no * ni;
        int rc = launch_gemm(g, S, st);
        if (rc != MLP_OK) return rc;
        const unsigned sblocks = (unsigned)(((int64_t)no * ni + SUM_COLS - 1) / SUM_COLS);
        hipLaunchKernelGGL(k_sum_parts, dim3(sblocks), dim3(THREADS), 0, st, (const float *)part, S,
                           (int64_t)no * ni, gW);
        // db_i[no] = sum_b dz[b][no]: row sums of the transposed gradient
        hipLaunchKernelGGL(k_rowsum, dim3(no), dim3(THREADS), 0, st, (const uint16_t *)dzT, ldt, gb);
        if (i == 0) break;
        // dz_prev[b][ni] = (sum_n dz[b][n] W_i[n][ni]) * gelu'(z_i[b][ni]), and its transposed
        // copy over dzT (whose last readers, the products above, come first on the stream).
        GemmArgs d{};
        d.a = dz;
        d.lda = no;
        d.b = hp(m, m->lay.wt[i]);
        d.ldb = no;
        d.M = batch;
        d.N = ni;
        d.K = no;
        d.mode = EPI_DGELU;
        d.c = hp(m, m->lay.dz[cur ^ 1]);
        d.ldc = ni;
        d.z = fp(m, m->lay.zf[i]);
        d.ct = dzT;
        d.ldt = ldt;
        rc = launch_gemm(d, 1, st);
        if (rc != MLP_OK) return rc;
        cur ^= 1;
    }
    return check();
}

int mlp_adam_step(mlp_t *m, float lr, float beta1, float beta2, float eps, void *stream) {
    if (!m || !(lr >= 0.0f) || !(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f) ||
        !(eps > 0.0f))
        return MLP_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    m->t += 1;
    const float bc1 = (float)(1.0 - pow((double)beta1, (double)m->t));
    const float bc2 = (float)(1.0 - pow((double)beta2, (double)m->t));
    const int64_t P = m->lay.P;
    BfMap bm{};
    bm.n = m->n;
    for (int i = 0; i < m->n; ++i) {
        bm.poff[i] = m->lay.poff[i];
        bm.no[i] = m->w[i + 1];
        bm.ni[i] = m->w[i];
        bm.wb[i] = hp(m, m->lay.wb[i]);
        bm.wt[i] = hp(m, m->lay.wt[i]);
    }
    hipLaunchKernelGGL(k_adam, dim3(nblocks(P)), dim3(THREADS), 0, st, fp(m, m->lay.params),
                       (const float *)fp(m, m->lay.grads), fp(m, m->lay.am), fp(m, m->lay.av), P, lr,
                       beta1, beta2, eps, bc1, bc2, bm);
    return check();
}

int mlp_train_step(mlp_t *m, const uint16_t *x, const float *target, int64_t batch, int n_valid,
                   float lr, float beta1, float beta2, float eps, float *y, float *loss,
                   void *stream) {
    if (!m || !x || !target || !y || !loss) return MLP_EINVAL;
    int rc = mlp_forward(m, x, y, batch, 1, stream);
    if (rc == MLP_OK) rc = mlp_mse(m, y, target, batch, n_valid, loss, stream);
    if (rc == MLP_OK) rc = mlp_backward(m, batch, stream);
    if (rc == MLP_OK) rc = mlp_adam_step(m, lr, beta1, beta2, eps, stream);
    return rc;
}

int mlp_gemm_nt(const uint16_t *a, int64_t lda, const uint16_t *b, int64_t ldb, const float *bias,
                int64_t M, int32_t N, int32_t K, int mode, void *c, int64_t ldc, float *z,
                void *stream) {
    if (!a || !b || !c || M < 1 || N < 1 || K < 8 || K % 8 != 0 || lda < K || ldb < K || ldc < N ||
        lda % 8 != 0 || ldb % 8 != 0 || (mode != EPI_F32 && mode != EPI_GELU))
        return MLP_EINVAL;
    GemmArgs g{};
    g.a = a;
    g.lda = lda;
    g.b = b;
    g.ldb = ldb;
    g.M = M;
    g.N = N;
    g.K = K;
    g.mode = mode;
    g.bias = bias;
    g.c = c;
    g.ldc = ldc;
    g.z = z;
    const int rc = launch_gemm(g, 1, (hipStream_t)stream);
    if (rc != MLP_OK) return rc;
    return check();
}

const char *mlp_strerror(int code) {
    switch (code) {
        case MLP_OK: return "ok";
        case MLP_EINVAL: return "invalid argument";
        case MLP_EHIP: return "HIP launch failure";
        default: return "unknown error";
    }
}

}  // extern "C"
