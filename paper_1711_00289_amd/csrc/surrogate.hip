// surrogate.hip -- kernels and host logic of the learned surrogate (include/surrogate.h): feature
// and target packing between the level-major column arrays and the network's row-major batches
// (transposed through LDS so both sides are accessed contiguously), per-feature statistics,
// normalisation, un-normalisation with the fallback test, and the gather / conv_step / scatter of
// the columns that fall back to the FP64 scheme.
#include <hip/hip_runtime.h>

#include <stdint.h>
#include <string.h>

#include <mutex>
#include <set>
#include <utility>

#include "conv.h"
#include "conv_internal.hpp"
#include "mlp.h"
#include "mlp_internal.hpp"
#include "surrogate.h"

using namespace cvk;

namespace {

constexpr int TB = 256;      // threads per block
constexpr int TC = 64;       // columns per transposing block
constexpr int WMAX = 256;    // widest feature row
constexpr int SPART = 256;   // row chunks of the statistics reduction

__device__ __forceinline__ uint16_t f2bf(float f) {  // round to nearest even
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

struct StateArgs {
    const double *T, *q, *pm;
    int64_t ld;
};

// Inputs of a block of TC columns into LDS as [feature][column] (normalised in mode 1), then out
// as rows.  mode 0: raw FP32 rows; mode 1: normalised BF16 rows.  With `vec` (row width a multiple
// of 8 and a 16-byte aligned output) each lane writes 8 BF16 or 4 FP32 features per store.
__global__ __launch_bounds__(TB) void k_pack_in(StateArgs s, int L, int64_t ncol, int w, int mode,
                                                const float *mean, const float *stdv, float *outf,
                                                uint16_t *outb, int vec) {
    extern __shared__ float sh[];  // [w][TC + 1]
    constexpr int SL = TC + 1;
    const int64_t c0 = (int64_t)blockIdx.x * TC;
    const int lane = threadIdx.x % TC, grp = threadIdx.x / TC;
    const int64_t c = c0 + lane;
    const int64_t ld = s.ld;
    // PU features per thread are loaded before any is converted, so that their loads are in
    // flight together instead of one round trip each.
    constexpr int PU = 8, G = TB / TC;
    for (int f0 = grp; f0 < w; f0 += G * PU) {
        double d[PU];
#pragma unroll
        for (int u = 0; u < PU; ++u) {
            const int f = f0 + u * G;
            d[u] = 0.0;
            if (c < ncol && f < 3 * L) {
                const double *src = f < L       ? s.T + (int64_t)f * ld
                                    : f < 2 * L ? s.q + (int64_t)(f - L) * ld
                                                : s.pm + (int64_t)(f - 2 * L) * ld;
                d[u] = __builtin_nontemporal_load(&src[c]);  // read once
            }
        }
#pragma unroll
        for (int u = 0; u < PU; ++u) {
            const int f = f0 + u * G;
            if (f >= w) break;
            float v = 0.0f;
            if (c < ncol && f < 3 * L) v = mode == 0 ? (float)d[u] : ((float)d[u] - mean[f]) / stdv[f];
            sh[f * SL + lane] = v;
        }
    }
    __syncthreads();
    const int nrows = (int)(ncol - c0 < TC ? ncol - c0 : TC);
    if (vec) {
        const int per = mode == 0 ? 4 : 8;  // features per 16-byte store
        const int cpr = w / per;
        for (int i = threadIdx.x; i < nrows * cpr; i += TB) {
            const int r = i / cpr, f0 = (i % cpr) * per;
            const int64_t o = (c0 + r) * w + f0;
            if (mode == 0) {
                *(float4 *)&outf[o] = make_float4(sh[f0 * SL + r], sh[(f0 + 1) * SL + r],
                                                  sh[(f0 + 2) * SL + r], sh[(f0 + 3) * SL + r]);
            } else {
                uint32_t h[4];
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    h[e] = (uint32_t)f2bf(sh[(f0 + 2 * e) * SL + r]) |
                           ((uint32_t)f2bf(sh[(f0 + 2 * e + 1) * SL + r]) << 16);
                *(uint4 *)&outb[o] = make_uint4(h[0], h[1], h[2], h[3]);
            }
        }
        return;
    }
    for (int i = threadIdx.x; i < nrows * w; i += TB) {
        const int r = i / w, f = i % w;
        const float v = sh[f * SL + r];
        const int64_t o = (c0 + r) * w + f;
        if (mode == 0) outf[o] = v;
        else outb[o] = f2bf(v);
    }
}

struct OutArgs {
    const double *dT_d, *dq_d, *pr_d, *dT_s, *dq_s, *pr_s;
    int64_t ld;
};

__global__ __launch_bounds__(TB) void k_pack_tgt(OutArgs a, int L, int64_t ncol, int w, float *out) {
    __shared__ float sh[WMAX][TC + 1];
    const int64_t c0 = (int64_t)blockIdx.x * TC;
    const int lane = threadIdx.x % TC, grp = threadIdx.x / TC;
    const int64_t c = c0 + lane;
    const int64_t ld = a.ld;
    for (int f = grp; f < w; f += TB / TC) {
        double v = 0.0;
        if (c < ncol) {
            if (f < L) v = a.dT_d[(int64_t)f * ld + c] + a.dT_s[(int64_t)f * ld + c];
            else if (f < 2 * L) v = a.dq_d[(int64_t)(f - L) * ld + c] + a.dq_s[(int64_t)(f - L) * ld + c];
            else if (f == 2 * L) v = a.pr_d[c] + a.pr_s[c];
        }
        sh[f][lane] = (float)v;
    }
    __syncthreads();
    const int64_t nrows = ncol - c0 < TC ? ncol - c0 : TC;
    for (int64_t i = threadIdx.x; i < nrows * w; i += TB) {
        const int r = (int)(i / w), f = (int)(i % w);
        out[(c0 + r) * w + f] = sh[f][r];
    }
}

// Statistics in two passes (the one-pass E[v^2] - E[v]^2 cancels for features that are nearly or
// exactly constant, such as the mid-level pressures of a grid with a common surface pressure).
// Pass p: block b sums, for 64 features (blockIdx.y selects them), the rows of chunk b -- v when
// center == NULL, else (v - center[j])^2 -- over four row groups combined in a fixed order.
__global__ __launch_bounds__(TB) void k_stats_part(const float *a, int64_t n, int w, int64_t chunk,
                                                   const double *center, double *part) {
    __shared__ double s1[TB / TC][TC];
    const int lane = threadIdx.x % TC, grp = threadIdx.x / TC;
    const int j = blockIdx.y * TC + lane;
    const int64_t r0 = (int64_t)blockIdx.x * chunk;
    const int64_t r1 = r0 + chunk < n ? r0 + chunk : n;
    double x1 = 0.0;
    if (j < w) {
        const double c = center ? center[j] : 0.0;
        for (int64_t r = r0 + grp; r < r1; r += TB / TC) {
            const double v = (double)a[r * w + j];
            x1 += center ? (v - c) * (v - c) : v;
        }
    }
    s1[grp][lane] = x1;
    __syncthreads();
    if (grp == 0 && j < w) {
        double t1 = 0.0;
        for (int g = 0; g < TB / TC; ++g) t1 += s1[g][lane];
        part[(int64_t)blockIdx.x * w + j] = t1;
    }
}

// Sum of the partials of feature j in order, divided by n, into out[j].
__global__ __launch_bounds__(TB) void k_stats_reduce(const double *part, int nparts, int64_t n, int w,
                                                     double *out) {
    const int j = blockIdx.x * TB + threadIdx.x;
    if (j >= w) return;
    double t = 0.0;
    for (int p = 0; p < nparts; ++p) t += part[(int64_t)p * w + j];
    out[j] = t / (double)n;
}

__global__ __launch_bounds__(TB) void k_stats_final(const double *mean, const double *var, int w,
                                                    int nvalid, float *meanf, float *stdf,
                                                    float *rmsf) {
    const int j = blockIdx.x * TB + threadIdx.x;
    if (j >= w) return;
    const double sd = var[j] > 0.0 ? sqrt(var[j]) : 0.0;
    meanf[j] = j < nvalid ? (float)mean[j] : 0.0f;
    stdf[j] = (j < nvalid && sd > 0.0) ? (float)sd : 1.0f;
    if (rmsf) rmsf[j] = (float)sqrt(var[j] + mean[j] * mean[j]);
}

__global__ __launch_bounds__(TB) void k_normalize(float *a, int64_t total, int w, const float *mean,
                                                  const float *stdv, uint16_t *outb) {
    const int64_t i = (int64_t)blockIdx.x * TB + threadIdx.x;
    if (i >= total) return;
    const int j = (int)(i % w);
    const float v = (a[i] - mean[j]) / stdv[j];
    if (outb) outb[i] = f2bf(v);
    else a[i] = v;
}

// Network output rows of TC columns -> level-major FP64 tendencies; flags columns whose predicted
// precipitation is outside [lo, hi] into the fallback list (first wavefront, one lane per column).
// With `vec` (row width a multiple of 4, 16-byte aligned rows) rows are read 4 outputs per load.
__global__ __launch_bounds__(TB) void k_unpack(const float *y, int L, int64_t ncol, int w,
                                               const float *mean, const float *stdv, double lo,
                                               double hi, double *dTdt, double *dqdt, double *prec,
                                               int64_t ld, int64_t col0, int *list, int *cnt, int vec) {
    extern __shared__ float sh[];  // [2L+1][TC + 1]
    constexpr int SL = TC + 1;
    const int64_t c0 = (int64_t)blockIdx.x * TC;
    const int nrows = (int)(ncol - c0 < TC ? ncol - c0 : TC);
    const int nf = 2 * L + 1;
    if (vec) {
        const int cpr = (nf + 3) / 4;  // f0 < nf <= w and w % 4 == 0, so f0 + 3 < w
        constexpr int UU = 4;          // 16-byte loads per thread in flight together
        for (int i0 = threadIdx.x; i0 < nrows * cpr; i0 += TB * UU) {
            float4 v[UU];
#pragma unroll
            for (int u = 0; u < UU; ++u) {
                const int i = i0 + u * TB;
                v[u] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
                if (i < nrows * cpr)
                    v[u] = *(const float4 *)&y[(c0 + i / cpr) * w + (i % cpr) * 4];
            }
#pragma unroll
            for (int u = 0; u < UU; ++u) {
                const int i = i0 + u * TB;
                if (i >= nrows * cpr) break;
                const int r = i / cpr, f0 = (i % cpr) * 4;
                const float e[4] = {v[u].x, v[u].y, v[u].z, v[u].w};
#pragma unroll
                for (int k = 0; k < 4; ++k)
                    if (f0 + k < nf) sh[(f0 + k) * SL + r] = e[k] * stdv[f0 + k] + mean[f0 + k];
            }
        }
    } else {
        for (int i = threadIdx.x; i < nrows * w; i += TB) {
            const int r = i / w, f = i % w;
            if (f < nf) sh[f * SL + r] = y[(c0 + r) * w + f] * stdv[f] + mean[f];
        }
    }
    __syncthreads();
    const int lane = threadIdx.x % TC, grp = threadIdx.x / TC;
    const int64_t c = c0 + lane;
    const bool live = lane < nrows;
    for (int f = grp; f < 2 * L; f += TB / TC) {
        if (!live) continue;
        const double v = (double)sh[f * SL + lane];
        if (f < L) __builtin_nontemporal_store(v, &dTdt[(int64_t)f * ld + col0 + c]);  // written once
        else __builtin_nontemporal_store(v, &dqdt[(int64_t)(f - L) * ld + col0 + c]);
    }
    if (grp == 0) {
        const double p = live ? (double)sh[2 * L * SL + lane] : 0.0;
        if (live) prec[col0 + c] = p > 0.0 ? p : 0.0;
        const bool fb = live && (p < lo || p > hi);
        const int slot = wave_append(fb, cnt);
        if (slot >= 0) list[slot] = (int)(col0 + c);
    }
}

// ------------------------------------------------------------------ fused inference
// The whole network for a tile of FR = 64 columns in one persistent block: the columns' features
// are packed (normalised, BF16) into an LDS activation tile [FR][FROW], every layer's product runs
// on the matrix cores (v_mfma_f32_32x32x16_bf16, FP32 accumulation) with its activations read
// from and written back to that tile, and the output layer is un-normalised and stored
// level-major, with the fallback test, straight from the accumulators.  No activation leaves the
// chip (the layer-by-layer path moves about 7 GB of them through HBM for the 884,736-column grid).
//
// Two blocks of four wavefronts share a CU (one wavefront of each on every SIMD) and run apart, so
// one block's epilogues (bias, GELU, BF16 rounding: vector ALU work) overlap the other's products
// on the matrix cores.  Hidden layers: wavefront w computes output columns [128 w, 128 w + 128) of
// all FR rows as the transposed product (weights as the first operand), so each lane ends with 4
// consecutive output columns of one row per accumulator group, written as one 8-byte LDS store.
// The output layer gives each wavefront one 32 x 32 tile.  Weight operands come straight from
// global memory (the network's 1.7 MB of BF16 weights stay in every XCD's L2) in a fragment-major
// copy (k_frag_pack), RING k-steps in flight; the next product's first RING steps are loaded
// before each epilogue, so they arrive while it runs.  Biases and normalisation statistics are
// kept in LDS.  Products accumulate K in steps of 16 in increasing order from zero, the bias is
// added in FP32, and GELU and the BF16 rounding are the layer-by-layer kernels', so the results
// are the same bits.
typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16;

constexpr int FR = 64;            // columns (network rows) per tile
constexpr int FH = 512;           // hidden width
constexpr int FIN = 96;           // input width
constexpr int FROW = FH + 8;      // BF16 per LDS row: the 16-byte pad puts the 32 rows a fragment
                                  // read serves on distinct 16-byte bank groups
constexpr int FWAVES = 4;
constexpr int FT = FWAVES * 64;
constexpr int FBLOCKS = 2;        // resident blocks per CU
constexpr int FN = FH / FWAVES;   // hidden output columns per wavefront
constexpr int FJ = FN / 32;       // 32-column weight tiles per wavefront
constexpr int FOUT = 64;          // output width
constexpr int RING = 3;           // k-steps of weight fragments in flight
constexpr int NSTH = FH / 16;     // k-steps of a 512-wide product
constexpr int NST0 = FIN / 16;    // k-steps of the input layer
constexpr size_t FACT = (size_t)FR * FROW * sizeof(uint16_t);  // activation tile bytes
constexpr size_t LDS_PER_CU = 160 * 1024;
static_assert(FR == 64 && FOUT == 64 && FWAVES == 4, "the output layer maps 2 x 2 tiles of 32 x 32 "
                                                      "onto the four wavefronts");
static_assert(RING <= NST0 && RING <= NSTH, "the weight ring fits every k-loop");

// LDS bytes of a block for a network of nl layers: the activation tile, then (float) the hidden
// layers' biases [nl - 1][FH], the output bias, scale and mean [FOUT] each, the input mean and
// scale [FIN] each.
size_t fused_lds(int nl) {
    return FACT + sizeof(float) * ((size_t)(nl - 1) * FH + 3 * FOUT + 2 * FIN);
}

struct FusedArgs {
    const double *T, *q, *pm;
    int64_t ld;
    int L;
    int64_t ncol, ntiles;
    int nl;                       // layers (hidden + output)
    const uint16_t *W[MLP_MAX_LAYERS];  // fragment-major BF16 weights (k_frag_pack)
    const float *B[MLP_MAX_LAYERS];
    const float *in_mean, *in_std, *out_mean, *out_std;
    double lo, hi;
    double *dTdt, *dqdt, *prec;   // level-major outputs with leading dimension ld
    int *list, *cnt;
};

// Layer l's weights (a wavefront-uniform selection among the kernel argument's entries, so the
// argument block is not copied to private memory for indexing).
__device__ __forceinline__ const uint16_t *layer_w(const FusedArgs &a, int l) {
    const uint16_t *p = a.W[0];
#pragma unroll
    for (int i = 1; i < MLP_MAX_LAYERS; ++i) p = l == i ? a.W[i] : p;
    return p;
}
__device__ __forceinline__ const float *layer_b(const FusedArgs &a, int l) {
    const float *p = a.B[0];
#pragma unroll
    for (int i = 1; i < MLP_MAX_LAYERS; ++i) p = l == i ? a.B[i] : p;
    return p;
}

// Weight fragments are read through a buffer resource (base and size in scalar registers): the
// per-step offsets are then constants in scalar registers next to one lane offset, not a 64-bit
// address per step and tile held in vector registers.  Reads past `bytes` return zeros.
typedef int i32x4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ __amdgpu_buffer_rsrc_t frag_rsrc(const uint16_t *w, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc((void *)w, 0, (int)bytes, 0x00020000);
}
__device__ __forceinline__ bf16x8 frag_load(__amdgpu_buffer_rsrc_t r, uint32_t voff,
                                            uint32_t soff) {
    return __builtin_bit_cast(bf16x8, __builtin_amdgcn_raw_buffer_load_b128(r, (int)voff,
                                                                             (int)soff, 0));
}

// Loads of the weight ring: slot q takes the fragments of k-step `st` of the wavefront's NJ tiles
// (TS bytes apart).  `sb` is an opaque zero: the offsets derived from it are formed where they are
// used instead of being hoisted, all of them, into registers for the whole kernel.
template <int NJ, uint32_t TS>
__device__ __forceinline__ void ring_load(bf16x8 (&bq)[RING][FJ], int q, __amdgpu_buffer_rsrc_t r,
                                          uint32_t woff, uint32_t sb, int st) {
#pragma unroll
    for (int j = 0; j < NJ; ++j) bq[q][j] = frag_load(r, woff, sb + j * TS + 1024u * st);
}
__device__ __forceinline__ uint32_t opaque_zero() {
    uint32_t z = 0;
    asm volatile("" : "+s"(z));
    return z;
}
template <int NJ, uint32_t TS>
__device__ __forceinline__ void ring_fill(bf16x8 (&bq)[RING][FJ], __amdgpu_buffer_rsrc_t r,
                                          uint32_t woff) {
    const uint32_t sb = opaque_zero();
#pragma unroll
    for (int q = 0; q < RING; ++q) ring_load<NJ, TS>(bq, q, r, woff, sb, q);
}

// The k-loop of a hidden product, fully unrolled: NS steps of 16 inputs, 2 row blocks x FJ
// weight tiles per wavefront.  The ring holds steps 0 .. RING - 1 on entry; the first step reads
// its activation fragments from LDS, each step reads the next step's before its products and
// loads the weight fragments RING steps ahead after them (the scheduler is kept from moving
// those loads).
template <int NS, int S = 0>
__device__ __forceinline__ void hidden_k(__amdgpu_buffer_rsrc_t r, uint32_t woff, uint32_t sb,
                                         const uint16_t *actK, f32x16 (&acc)[2][FJ],
                                         bf16x8 (&bq)[RING][FJ], bf16x8 (&af)[2][2]) {
    if constexpr (S < NS) {
        constexpr int slot = S % RING, cur = S % 2;
        if constexpr (S == 0) {
#pragma unroll
            for (int rb = 0; rb < 2; ++rb) af[0][rb] = *(const bf16x8 *)(actK + 32 * rb * FROW);
        }
        if constexpr (S + 1 < NS) {
#pragma unroll
            for (int rb = 0; rb < 2; ++rb)
                af[cur ^ 1][rb] = *(const bf16x8 *)(actK + 32 * rb * FROW + 16 * (S + 1));
        }
#pragma unroll
        for (int j = 0; j < FJ; ++j)
#pragma unroll
            for (int rb = 0; rb < 2; ++rb)
                acc[rb][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                    bq[slot][j], af[cur][rb], S == 0 ? f32x16{} : acc[rb][j], 0, 0, 0);
        if constexpr (S + RING < NS) ring_load<FJ, NS * 1024u>(bq, slot, r, woff, sb, S + RING);
        __builtin_amdgcn_sched_barrier(0);
        hidden_k<NS, S + 1>(r, woff, sb, actK, acc, bq, af);
    }
}

// The output layer's k-loop for the wavefront's 32 x 32 tile (ring slot column 0).
template <int S = 0>
__device__ __forceinline__ void out_k(__amdgpu_buffer_rsrc_t r, uint32_t woff, uint32_t sb,
                                      const uint16_t *actK, f32x16 &acc, bf16x8 (&bq)[RING][FJ],
                                      bf16x8 (&af)[2][2]) {
    if constexpr (S < NSTH) {
        constexpr int slot = S % RING, cur = S % 2;
        if constexpr (S == 0) af[0][0] = *(const bf16x8 *)actK;
        if constexpr (S + 1 < NSTH) af[cur ^ 1][0] = *(const bf16x8 *)(actK + 16 * (S + 1));
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(bq[slot][0], af[cur][0],
                                                      S == 0 ? f32x16{} : acc, 0, 0, 0);
        if constexpr (S + RING < NSTH) ring_load<1, 0>(bq, slot, r, woff, sb, S + RING);
        __builtin_amdgcn_sched_barrier(0);
        out_k<S + 1>(r, woff, sb, actK, acc, bq, af);
    }
}

// The epilogue of a hidden product as groups of 4 elements: group gi is row block gi / 16,
// weight tile (gi / 4) % 4, accumulator registers 4 (gi % 4) .. + 3 (4 consecutive columns of one
// row in the transposed layout).  `bias` (LDS) and `dst` point at the lane's first column.  Each
// group reads the next group's biases before its own arithmetic, and the scheduler is kept from
// pulling every group's reads to the front (which would hold them all in registers).
template <int GI>
__device__ __forceinline__ float4 epi_bias(const float *bias) {
    return *(const float4 *)(bias + 32 * ((GI / 4) % FJ) + 8 * (GI % 4));
}
template <int GI, int GN>
__device__ __forceinline__ void epi_groups(const f32x16 (&acc)[2][FJ], const float *bias,
                                           uint16_t *dst, float4 b) {
    if constexpr (GI < GN) {
        constexpr int rb = GI / 16, j = (GI / 4) % FJ, g = GI % 4;
        float4 bn = b;
        if constexpr (GI + 1 < GN) bn = epi_bias<GI + 1>(bias);
        const float y0 = mlpk::gelu(acc[rb][j][4 * g + 0] + b.x);
        const float y1 = mlpk::gelu(acc[rb][j][4 * g + 1] + b.y);
        const float y2 = mlpk::gelu(acc[rb][j][4 * g + 2] + b.z);
        const float y3 = mlpk::gelu(acc[rb][j][4 * g + 3] + b.w);
        *(uint2 *)(dst + 32 * rb * FROW + 32 * j + 8 * g) =
            make_uint2(mlpk::bf16x2(y0, y1), mlpk::bf16x2(y2, y3));
        __builtin_amdgcn_sched_barrier(0);
        epi_groups<GI + 1, GN>(acc, bias, dst, bn);
    }
}

__global__ __launch_bounds__(FT, FBLOCKS) void k_surr_fused(FusedArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    uint16_t *act = (uint16_t *)smem;  // [FR][FROW]
    float *pb = (float *)(smem + FACT);
    float *p_hb = pb;                              // hidden biases [nl - 1][FH]
    float *p_ob = p_hb + (a.nl - 1) * FH;          // output bias, scale, mean [FOUT] each
    float *p_os = p_ob + FOUT, *p_om = p_os + FOUT;
    float *p_im = p_om + FOUT, *p_is = p_im + FIN; // input mean, scale [FIN] each
    const int tid = threadIdx.x;
    const int lane = tid % 64;
    const int wu = __builtin_amdgcn_readfirstlane(tid / 64);  // the wavefront index, uniform
    const int lrow = lane & 31, lk = 8 * (lane >> 5);
    const int L = a.L;
    for (int i = tid; i < (a.nl - 1) * FH; i += FT) p_hb[i] = layer_b(a, i / FH)[i % FH];
    for (int i = tid; i < FOUT; i += FT) {
        p_ob[i] = layer_b(a, a.nl - 1)[i];
        p_os[i] = a.out_std[i];
        p_om[i] = a.out_mean[i];
    }
    for (int i = tid; i < FIN; i += FT) {
        p_im[i] = a.in_mean[i];
        p_is[i] = a.in_std[i];
    }
    // Lane-fixed LDS positions and weight offsets.
    const uint16_t *actK = act + lrow * FROW + lk;
    uint16_t *dst = act + lrow * FROW + FN * wu + 4 * (lane >> 5);
    const uint32_t woff0 = (uint32_t)(FJ * wu) * (NST0 * 1024u) + 16u * lane;
    const uint32_t woffH = (uint32_t)(FJ * wu) * (NSTH * 1024u) + 16u * lane;
    const int orb = wu % 2, ont = wu / 2;  // the output tile
    const uint32_t woffO = (uint32_t)ont * (NSTH * 1024u) + 16u * lane;
    // Buffer resources of the layers' fragment-major weights.
    auto rsrc = [&](int l) {
        const uint32_t bytes = l == 0 ? FIN * FH * 2u : l + 1 < a.nl ? FH * FH * 2u : FH * FOUT * 2u;
        return frag_rsrc(layer_w(a, l), bytes);
    };
    const __amdgpu_buffer_rsrc_t r0 = rsrc(0), rO = rsrc(a.nl - 1);
    bf16x8 bq[RING][FJ], af[2][2];
    f32x16 acc[2][FJ], accO;
    double d[3][8];

    // Pack, in two halves: `pack_load` puts tile t's features in registers (task k of wavefront
    // w is feature group w + 4 k, 8 levels of the lane's column, contiguous across the wavefront
    // and in flight together); `pack_store` normalises them, rounds to BF16 and writes one
    // 16-byte row piece per group.  Features past 3L and rows past the grid are zero.
    auto pack_load = [&](int64_t t) {
        int64_t ld = a.ld;
        int pl = lane, pw = wu;
        asm volatile("" : "+s"(ld), "+v"(pl), "+s"(pw));  // recomputed per tile, not hoisted
        const int64_t col = t * FR + pl;
        const bool rok = col < a.ncol;
        static_assert(FIN / 8 == 3 * FWAVES, "three feature groups per wavefront");
#pragma unroll
        for (int k = 0; k < 3; ++k) {
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int f = 8 * (pw + FWAVES * k) + e;  // wavefront-uniform
                const double *src = f < L       ? a.T + (int64_t)f * ld
                                    : f < 2 * L ? a.q + (int64_t)(f - L) * ld
                                                : a.pm + (int64_t)(f - 2 * L) * ld;
                d[k][e] = f < 3 * L && rok ? __builtin_nontemporal_load(&src[col]) : 0.0;
            }
        }
    };
    auto pack_store = [&]() {
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const int g = wu + FWAVES * k;
            float v[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int f = 8 * g + e;
                v[e] = ((float)d[k][e] - p_im[f]) / p_is[f];
                v[e] = f < 3 * L ? v[e] : 0.0f;  // d is 0 past the grid: (0 - mean) / scale
            }
            *(uint4 *)&act[lane * FROW + 8 * g] =
                make_uint4(mlpk::bf16x2(v[0], v[1]), mlpk::bf16x2(v[2], v[3]),
                           mlpk::bf16x2(v[4], v[5]), mlpk::bf16x2(v[6], v[7]));
        }
    };

    int64_t tile = blockIdx.x;  // the grid is at most the number of tiles
    ring_fill<FJ, NST0 * 1024u>(bq, r0, woff0);
    pack_load(tile);
    __syncthreads();  // parameters in LDS
    pack_store();
    for (;;) {
        const int64_t c0 = tile * FR;  // rows past the grid are computed and not stored
        __syncthreads();
        // Hidden layers.  The ring holds the first steps of layer l's fragments on entry.
        for (int l = 0; l + 1 < a.nl; ++l) {
            if (l == 0) {
                hidden_k<NST0>(r0, woff0, opaque_zero(), actK, acc, bq, af);
            } else {
                hidden_k<NSTH>(rsrc(l), woffH, opaque_zero(), actK, acc, bq, af);
            }
            // The next product's first steps, in flight during the epilogue.
            if (l + 2 < a.nl) {
                ring_fill<FJ, NSTH * 1024u>(bq, rsrc(l + 1), woffH);
            } else {
                ring_fill<1, 0>(bq, rO, woffO);
            }
            __syncthreads();  // every wavefront has read the layer's inputs
            const float *bias = p_hb + l * FH + FN * wu + 4 * (lane >> 5);
            epi_groups<0, 8 * FJ>(acc, bias, dst, epi_bias<0>(bias));
            __syncthreads();
        }
        // Output layer: wavefront w's tile is rows 32 (w % 2) .., outputs 32 (w / 2) ...
        out_k(rO, woffO, opaque_zero(), actK + 32 * orb * FROW, accO, bq, af);
        ring_fill<FJ, NST0 * 1024u>(bq, r0, woff0);  // the next tile's first product
        const int64_t next = tile + gridDim.x;
        const bool have = next < a.ntiles;
        pack_load(next);  // in flight while the outputs are stored (nothing past the grid)
        {
            // Un-normalise and store (transposed layout: register r of lane l is output
            // 32 nt + 8 (r / 4) + 4 (l / 32) + r % 4 of column c0 + 32 rb + l % 32); tendencies
            // level-major, precipitation clipped at zero, and the fallback test on it.
            int64_t ld = a.ld;
            int pl = lane;
            asm volatile("" : "+s"(ld), "+v"(pl));  // recomputed per tile, not hoisted
            const int64_t col = c0 + 32 * orb + (pl & 31);
            const bool live = col < a.ncol;
            bool fb = false;
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int f = 32 * ont + 8 * (r >> 2) + 4 * (pl >> 5) + (r & 3);
                if (f > 2 * L) continue;
                const float y = accO[r] + p_ob[f];
                const double v = (double)(y * p_os[f] + p_om[f]);
                if (f < L) {
                    if (live) __builtin_nontemporal_store(v, &a.dTdt[(int64_t)f * ld + col]);
                } else if (f < 2 * L) {
                    if (live) __builtin_nontemporal_store(v, &a.dqdt[(int64_t)(f - L) * ld + col]);
                } else {
                    if (live) a.prec[col] = v > 0.0 ? v : 0.0;
                    fb = live && (v < a.lo || v > a.hi);
                }
            }
            const int slot = wave_append(fb, a.cnt);
            if (slot >= 0) a.list[slot] = (int)col;
        }
        if (!have) break;
        __syncthreads();  // every wavefront has read the tile before it is repacked
        pack_store();
        tile = next;
    }
}

// Fragment-major copy of one layer's BF16 weights W [N][K] for the fused kernel: the fragment of
// n-tile t (32 output columns) at k-step s (16 inputs) is the MFMA operand as the 64 lanes hold it
// (lane i: row 32 t + i % 32, inputs 16 s + 8 (i / 32) .. + 7), stored as 64 consecutive 16-byte
// pieces at ((t * K / 16 + s) * 64 + i) * 8.
__global__ __launch_bounds__(TB) void k_frag_pack(const uint16_t *W, int N, int K, uint16_t *dst) {
    const int64_t g = (int64_t)blockIdx.x * TB + threadIdx.x;
    const int S = K / 16;
    if (g >= (int64_t)(N / 32) * S * 64) return;
    const int i = (int)(g % 64);
    const int64_t ts = g / 64;
    const int t = (int)(ts / S), st = (int)(ts % S);
    const uint16_t *src = W + (int64_t)(32 * t + i % 32) * K + 16 * st + 8 * (i / 32);
    *(uint4 *)(dst + g * 8) = *(const uint4 *)src;
}

struct Compact {
    double *T, *q, *pm, *z, *pi, *phis, *pblh, *tke;
    int64_t ld;
};

__global__ __launch_bounds__(TB) void k_gather(conv_state_t s, int L, const int *list, const int *cnt,
                                               Compact d) {
    const int64_t i = (int64_t)blockIdx.x * TB + threadIdx.x;
    if (i >= *cnt) return;
    const int64_t c = list[i];
    const int64_t ls = s.ld, lc = d.ld;
    for (int k = 0; k < L; ++k) {
        d.T[k * lc + i] = s.T[k * ls + c];
        d.q[k * lc + i] = s.q[k * ls + c];
        d.pm[k * lc + i] = s.p_mid[k * ls + c];
        d.z[k * lc + i] = s.z[k * ls + c];
    }
    for (int k = 0; k <= L; ++k) d.pi[k * lc + i] = s.p_int[k * ls + c];
    d.phis[i] = s.phis[c];
    d.pblh[i] = s.pblh[c];
    d.tke[i] = s.tke[c];
}

__global__ __launch_bounds__(TB) void k_scatter(conv_deep_out_t dd, conv_shallow_out_t ss, int64_t lc,
                                                int L, const int *list, const int *cnt, double *dTdt,
                                                double *dqdt, double *prec, int64_t ld) {
    const int64_t i = (int64_t)blockIdx.x * TB + threadIdx.x;
    if (i >= *cnt) return;
    const int64_t c = list[i];
    for (int k = 0; k < L; ++k) {
        dTdt[k * ld + c] = dd.dTdt[k * lc + i] + ss.dTdt[k * lc + i];
        dqdt[k * ld + c] = dd.dqdt[k * lc + i] + ss.dqdt[k * lc + i];
    }
    prec[c] = dd.prec[i] + ss.prec[i];
}

__global__ void k_zero_int(int *p) {
    if (threadIdx.x == 0) p[0] = 0;
}

unsigned nb(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

bool al16(const void *p) { return ((uintptr_t)p & 15u) == 0; }
size_t pack_lds(int w) { return (size_t)w * (TC + 1) * sizeof(float); }
size_t unpack_lds(int L) { return (size_t)(2 * L + 1) * (TC + 1) * sizeof(float); }

// Allows `bytes` of dynamic LDS for `fn` on the current device (above 64 KiB a function attribute
// must be raised; done once per device and kernel).
int lds_limit(const void *fn, size_t bytes) {
    if (bytes <= 65536) return CONV_OK;
    static std::mutex mu;
    static std::set<std::pair<int, const void *>> done;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return CONV_EHIP;
    std::lock_guard<std::mutex> g(mu);
    if (done.count({dev, fn})) return CONV_OK;
    if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024) != hipSuccess)
        return CONV_EHIP;
    done.insert({dev, fn});
    return CONV_OK;
}
size_t al(size_t x) { return (x + 255) & ~size_t(255); }

// Networks the fused inference kernel handles: an input of FIN features holding the 3L packed
// features, hidden layers of width FH, an output of FOUT holding 2L + 1, and few enough layers
// that two blocks' LDS (activation tile and parameters) fit a CU.
bool fused_ok(const mlpk::NetView &v, int L) {
    if (v.n < 2 || v.w[0] != FIN || 3 * L > FIN) return false;
    if (v.w[v.n] != FOUT || 2 * L + 1 > FOUT) return false;
    for (int i = 1; i < v.n; ++i)
        if (v.w[i] != FH) return false;
    return FBLOCKS * fused_lds(v.n) <= LDS_PER_CU;
}

struct SLayout {
    size_t x, y, norm, list, cnt, wfrag, cst, dout, sout, cws, total;
    size_t cws_bytes;
};

SLayout surr_layout(int L, int w_in, int w_out, int64_t maxc, int64_t chunk, int cus) {
    SLayout l{};
    size_t off = 0;
    auto take = [&](size_t b) {
        const size_t o = off;
        off = al(off + b);
        return o;
    };
    const size_t m = (size_t)maxc;
    l.x = take((size_t)chunk * w_in * 2);
    l.y = take((size_t)chunk * w_out * 4);
    l.norm = take((size_t)2 * (w_in + w_out) * 4);
    l.list = take(m * 4);
    l.cnt = take(256);
    l.wfrag = take((size_t)MLP_MAX_LAYERS * FH * FH * sizeof(uint16_t));
    l.cst = take(((size_t)4 * L + (L + 1) + 3) * m * 8);
    l.dout = take(((size_t)2 * L + 2 * (L + 1) + 2) * m * 8 + 4 * m * 4);
    l.sout = take(((size_t)2 * L + (L + 1) + 2) * m * 8 + 3 * m * 4);
    (void)cus;
    l.cws_bytes = conv_workspace_bytes(maxc, L);
    l.cws = take(l.cws_bytes);
    l.total = off;
    return l;
}

int hip_err() {
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? CONV_OK : CONV_EHIP;
}

}  // namespace

struct surr {
    mlp_t *net;
    int L, w_in, w_out;
    int64_t maxc, chunk;
    conv_params_t P;
    char *ws;
    SLayout lay;
    double lo, hi;
    int fused = 1;  // surr_set_fused
};

namespace {

float *nrm(surr *s, int which) {  // 0 in_mean, 1 in_std, 2 out_mean, 3 out_std
    float *b = (float *)(s->ws + s->lay.norm);
    switch (which) {
        case 0: return b;
        case 1: return b + s->w_in;
        case 2: return b + 2 * s->w_in;
        default: return b + 2 * s->w_in + s->w_out;
    }
}

}  // namespace

extern "C" {

int surr_pack_inputs_raw(const conv_state_t *s, int32_t nlev, int64_t ncol, int32_t w_in,
                         float *out, void *stream) {
    if (!s || !s->T || !s->q || !s->p_mid || !out || nlev < 2 || ncol < 0 || w_in < 3 * nlev ||
        w_in > WMAX || s->ld < ncol)
        return CONV_EINVAL;
    if (ncol == 0) return CONV_OK;
    StateArgs a{s->T, s->q, s->p_mid, s->ld};
    if (lds_limit((const void *)k_pack_in, pack_lds(w_in)) != CONV_OK) return CONV_EHIP;
    hipLaunchKernelGGL(k_pack_in, dim3(nb(ncol, TC)), dim3(TB), pack_lds(w_in), (hipStream_t)stream, a,
                       nlev, ncol, w_in, 0, (const float *)nullptr, (const float *)nullptr, out,
                       (uint16_t *)nullptr, (int)(w_in % 4 == 0 && al16(out)));
    return hip_err();
}

int surr_pack_inputs(const conv_state_t *s, int32_t nlev, int64_t ncol, int32_t w_in,
                     const float *mean, const float *std, uint16_t *x, void *stream) {
    if (!s || !s->T || !s->q || !s->p_mid || !x || !mean || !std || nlev < 2 || ncol < 0 ||
        w_in < 3 * nlev || w_in > WMAX || s->ld < ncol)
        return CONV_EINVAL;
    if (ncol == 0) return CONV_OK;
    StateArgs a{s->T, s->q, s->p_mid, s->ld};
    if (lds_limit((const void *)k_pack_in, pack_lds(w_in)) != CONV_OK) return CONV_EHIP;
    hipLaunchKernelGGL(k_pack_in, dim3(nb(ncol, TC)), dim3(TB), pack_lds(w_in), (hipStream_t)stream, a,
                       nlev, ncol, w_in, 1, mean, std, (float *)nullptr, x,
                       (int)(w_in % 8 == 0 && al16(x)));
    return hip_err();
}

int surr_pack_targets_raw(const conv_deep_out_t *d, const conv_shallow_out_t *sh, int32_t nlev,
                          int64_t ld, int64_t ncol, int32_t w_out, float *out, void *stream) {
    if (!d || !sh || !d->dTdt || !d->dqdt || !d->prec || !sh->dTdt || !sh->dqdt || !sh->prec || !out ||
        nlev < 2 || ncol < 0 || ld < ncol || w_out < 2 * nlev + 1 || w_out > WMAX)
        return CONV_EINVAL;
    if (ncol == 0) return CONV_OK;
    OutArgs a{d->dTdt, d->dqdt, d->prec, sh->dTdt, sh->dqdt, sh->prec, ld};
    hipLaunchKernelGGL(k_pack_tgt, dim3(nb(ncol, TC)), dim3(TB), 0, (hipStream_t)stream, a, nlev, ncol,
                       w_out, out);
    return hip_err();
}

size_t surr_col_stats_scratch_bytes(int32_t w) {
    return (w < 1 || w > WMAX) ? 0 : ((size_t)SPART * w + 2 * (size_t)w) * sizeof(double);
}

int surr_col_stats(const float *a, int64_t n, int32_t w, int32_t n_valid, float *mean, float *std,
                   float *rms, void *scratch, size_t scratch_bytes, void *stream) {
    if (!a || !mean || !std || !scratch || n < 1 || w < 1 || w > WMAX || n_valid < 0 || n_valid > w ||
        scratch_bytes < surr_col_stats_scratch_bytes(w))
        return CONV_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    const int64_t chunk = (n + SPART - 1) / SPART;
    const int parts = (int)((n + chunk - 1) / chunk);
    double *part = (double *)scratch;
    double *m64 = part + (size_t)SPART * w;
    double *v64 = m64 + w;
    const dim3 grid(parts, nb(w, TC));
    hipLaunchKernelGGL(k_stats_part, grid, dim3(TB), 0, st, a, n, w, chunk, (const double *)nullptr, part);
    hipLaunchKernelGGL(k_stats_reduce, dim3(nb(w, TB)), dim3(TB), 0, st, (const double *)part, parts, n, w,
                       m64);
    hipLaunchKernelGGL(k_stats_part, grid, dim3(TB), 0, st, a, n, w, chunk, (const double *)m64, part);
    hipLaunchKernelGGL(k_stats_reduce, dim3(nb(w, TB)), dim3(TB), 0, st, (const double *)part, parts, n, w,
                       v64);
    hipLaunchKernelGGL(k_stats_final, dim3(nb(w, TB)), dim3(TB), 0, st, (const double *)m64,
                       (const double *)v64, w, n_valid, mean, std, rms);
    return hip_err();
}

int surr_normalize(float *a, int64_t n, int32_t w, const float *mean, const float *std,
                   uint16_t *out_bf16, void *stream) {
    if (!a || !mean || !std || n < 0 || w < 1) return CONV_EINVAL;
    if (n == 0) return CONV_OK;
    hipLaunchKernelGGL(k_normalize, dim3(nb(n * w, TB)), dim3(TB), 0, (hipStream_t)stream, a, n * w, w,
                       mean, std, out_bf16);
    return hip_err();
}

size_t surr_workspace_bytes(int32_t nlev, int32_t w_in, int32_t w_out, int64_t max_cols,
                            int64_t chunk) {
    if (nlev < 2 || w_in < 3 * nlev || w_in > WMAX || w_out < 2 * nlev + 1 || w_out > WMAX ||
        max_cols < 1 || max_cols > INT32_MAX || chunk < 1)
        return 0;
    return surr_layout(nlev, w_in, w_out, max_cols, chunk, device_cus()).total;
}

int surr_create(mlp_t *net, int32_t nlev, int32_t w_in, int32_t w_out, int64_t max_cols,
                int64_t chunk, const conv_params_t *params, void *workspace, size_t ws_bytes,
                surr_t **out) {
    if (!net || !params || !workspace || !out || nlev < 2 || w_in < 3 * nlev || w_in > WMAX ||
        w_out < 2 * nlev + 1 || w_out > WMAX || max_cols < 1 || max_cols > INT32_MAX || chunk < 1)
        return CONV_EINVAL;
    if (((uintptr_t)workspace & 255u) != 0) return CONV_EINVAL;
    const SLayout l = surr_layout(nlev, w_in, w_out, max_cols, chunk, device_cus());
    if (ws_bytes < l.total || l.cws_bytes == 0) return CONV_EINVAL;
    surr *s = new surr;
    s->net = net;
    s->L = nlev;
    s->w_in = w_in;
    s->w_out = w_out;
    s->maxc = max_cols;
    s->chunk = chunk;
    s->P = *params;
    s->ws = (char *)workspace;
    s->lay = l;
    s->lo = 0.0;
    s->hi = 0.0;
    *out = s;
    return CONV_OK;
}

void surr_destroy(surr_t *s) { delete s; }

int surr_set_fused(surr_t *s, int enable) {
    if (!s) return CONV_EINVAL;
    s->fused = enable != 0;
    return s->fused && fused_ok(mlpk::net_view(s->net), s->L) ? 1 : 0;
}

int surr_set_norm(surr_t *s, const float *in_mean, const float *in_std, const float *out_mean,
                  const float *out_std, double prec_lo, double prec_hi, void *stream) {
    if (!s || !in_mean || !in_std || !out_mean || !out_std || !(prec_lo <= prec_hi)) return CONV_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    const float *src[4] = {in_mean, in_std, out_mean, out_std};
    const int len[4] = {s->w_in, s->w_in, s->w_out, s->w_out};
    for (int i = 0; i < 4; ++i)
        if (hipMemcpyAsync(nrm(s, i), src[i], len[i] * sizeof(float), hipMemcpyDeviceToDevice, st) !=
            hipSuccess)
            return CONV_EHIP;
    s->lo = prec_lo;
    s->hi = prec_hi;
    return CONV_OK;
}

int surr_infer(surr_t *s, const conv_state_t *state, int64_t ncol, double *dTdt, double *dqdt,
               double *prec, int fallback, int64_t *n_fallback, void *stream) {
    if (!s || !state || !state->T || !state->q || !state->p_mid || !dTdt || !dqdt || !prec ||
        ncol < 0 || ncol > s->maxc || state->ld < ncol)
        return CONV_EINVAL;
    if (fallback && (!state->z || !state->p_int || !state->phis || !state->pblh || !state->tke))
        return CONV_EINVAL;
    if (ncol == 0) {
        if (fallback && n_fallback) *n_fallback = 0;
        return CONV_OK;
    }
    hipStream_t st = (hipStream_t)stream;
    const int L = s->L;
    const int64_t ld = state->ld;
    uint16_t *X = (uint16_t *)(s->ws + s->lay.x);
    float *Y = (float *)(s->ws + s->lay.y);
    int *list = (int *)(s->ws + s->lay.list);
    int *cnt = (int *)(s->ws + s->lay.cnt);
    if (lds_limit((const void *)k_pack_in, pack_lds(s->w_in)) != CONV_OK ||
        lds_limit((const void *)k_unpack, unpack_lds(L)) != CONV_OK)
        return CONV_EHIP;
    hipLaunchKernelGGL(k_zero_int, dim3(1), dim3(64), 0, st, cnt);
    const mlpk::NetView nv = mlpk::net_view(s->net);
    const bool fused = s->fused && fused_ok(nv, L);
    if (fused) {
        // The whole network per tile on the chip: one launch for every column, no chunks.
        if (lds_limit((const void *)k_surr_fused, fused_lds(nv.n)) != CONV_OK) return CONV_EHIP;
        FusedArgs fa{};
        fa.T = state->T;
        fa.q = state->q;
        fa.pm = state->p_mid;
        fa.ld = ld;
        fa.L = L;
        fa.ncol = ncol;
        fa.ntiles = (ncol + FR - 1) / FR;
        fa.nl = nv.n;
        uint16_t *wf = (uint16_t *)(s->ws + s->lay.wfrag);
        for (int i = 0; i < nv.n; ++i) {
            const int64_t cnt_i = (int64_t)nv.w[i + 1] * nv.w[i];
            hipLaunchKernelGGL(k_frag_pack, dim3((unsigned)nb(cnt_i / 8, TB)), dim3(TB), 0, st,
                               nv.wb[i], nv.w[i + 1], nv.w[i], wf);
            fa.W[i] = wf;
            fa.B[i] = nv.bias[i];
            wf += cnt_i;
        }
        fa.in_mean = nrm(s, 0);
        fa.in_std = nrm(s, 1);
        fa.out_mean = nrm(s, 2);
        fa.out_std = nrm(s, 3);
        fa.lo = s->lo;
        fa.hi = s->hi;
        fa.dTdt = dTdt;
        fa.dqdt = dqdt;
        fa.prec = prec;
        fa.list = list;
        fa.cnt = cnt;
        const int64_t slots = (int64_t)FBLOCKS * device_cus();
        const int64_t grid = fa.ntiles < slots ? fa.ntiles : slots;
        hipLaunchKernelGGL(k_surr_fused, dim3((unsigned)grid), dim3(FT), fused_lds(nv.n), st, fa);
    }
    for (int64_t c0 = 0; c0 < ncol && !fused; c0 += s->chunk) {
        const int64_t n = ncol - c0 < s->chunk ? ncol - c0 : s->chunk;
        StateArgs a{state->T + c0, state->q + c0, state->p_mid + c0, ld};
        hipLaunchKernelGGL(k_pack_in, dim3(nb(n, TC)), dim3(TB), pack_lds(s->w_in), st, a, L, n,
                           s->w_in, 1, (const float *)nrm(s, 0), (const float *)nrm(s, 1),
                           (float *)nullptr, X, (int)(s->w_in % 8 == 0));
        const int rc = mlp_forward(s->net, X, Y, n, 0, stream);
        if (rc != MLP_OK) return rc == MLP_EINVAL ? CONV_EINVAL : CONV_EHIP;
        hipLaunchKernelGGL(k_unpack, dim3(nb(n, TC)), dim3(TB), unpack_lds(L), st, (const float *)Y, L,
                           n, s->w_out, (const float *)nrm(s, 2), (const float *)nrm(s, 3), s->lo,
                           s->hi, dTdt, dqdt, prec, ld, c0, list, cnt, (int)(s->w_out % 4 == 0));
    }
    if (hip_err() != CONV_OK) return CONV_EHIP;
    if (!fallback) return CONV_OK;
    int nfb = 0;
    if (hipMemcpyAsync(&nfb, cnt, sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return CONV_EHIP;
    if (n_fallback) *n_fallback = nfb;
    if (nfb == 0) return CONV_OK;
    const int64_t m = s->maxc;
    double *cb = (double *)(s->ws + s->lay.cst);
    Compact cs{cb, cb + (int64_t)L * m, cb + (int64_t)2 * L * m, cb + (int64_t)3 * L * m,
               cb + (int64_t)4 * L * m, cb + (int64_t)(5 * L + 1) * m, cb + (int64_t)(5 * L + 2) * m,
               cb + (int64_t)(5 * L + 3) * m, m};
    hipLaunchKernelGGL(k_gather, dim3(nb(nfb, TB)), dim3(TB), 0, st, *state, L, (const int *)list,
                       (const int *)cnt, cs);
    double *db = (double *)(s->ws + s->lay.dout);
    int32_t *di = (int32_t *)(db + ((int64_t)2 * L + 2 * (L + 1) + 2) * m);
    conv_deep_out_t dd{db, db + (int64_t)L * m, db + (int64_t)2 * L * m, db + (int64_t)(3 * L + 1) * m,
                       db + (int64_t)(4 * L + 2) * m, db + (int64_t)(4 * L + 3) * m, di, di + m,
                       di + 2 * m, di + 3 * m};
    double *sb = (double *)(s->ws + s->lay.sout);
    int32_t *si = (int32_t *)(sb + ((int64_t)2 * L + (L + 1) + 2) * m);
    conv_shallow_out_t ss{sb, sb + (int64_t)L * m, sb + (int64_t)2 * L * m, sb + (int64_t)(3 * L + 1) * m,
                          sb + (int64_t)(3 * L + 2) * m, si, si + m, si + 2 * m};
    conv_state_t cst{cs.T, cs.q, cs.pm, cs.z, cs.pi, cs.phis, cs.pblh, cs.tke, m, state->dt};
    conv_ctx_t *ctx = nullptr;
    int rc = conv_create(nfb, L, &s->P, s->ws + s->lay.cws, s->lay.cws_bytes, &ctx);
    if (rc != CONV_OK) return rc;
    rc = conv_step(ctx, &cst, &dd, &ss, stream);
    conv_destroy(ctx);
    if (rc != CONV_OK) return rc;
    hipLaunchKernelGGL(k_scatter, dim3(nb(nfb, TB)), dim3(TB), 0, st, dd, ss, m, L, (const int *)list,
                       (const int *)cnt, dTdt, dqdt, prec, ld);
    return hip_err();
}

}  // extern "C"
