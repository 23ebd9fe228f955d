// conv_internal.hpp -- types and helpers shared by the library's translation units (forward
// kernels in conv.hip, adjoint kernels in conv_adjoint.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include "conv.h"
#include "conv_physics.hpp"

namespace cvk {

constexpr int BLOCK = 256;
constexpr int WAVE = 64;
constexpr int NWAVES = BLOCK / WAVE;
constexpr int NCOUNTERS = 64;

// One grid of columns with its arrays and parameters.
struct Member {
    const double *T, *q, *pm, *pi, *z, *phis, *pblh, *tke;
    int64_t ld;
    double dt;
    int64_t ncol;
    int64_t tile0;  // first tile of this member in the launch's tile space
    int nlev, pad_;
    conv_params_t P;
    conv_deep_out_t dout;
    conv_shallow_out_t sout;
};

// Pointers read from device memory (the ensemble's member table) are generic to the compiler:
// loads and stores through them become FLAT instructions, which cannot take a scalar base and
// also count against the LDS/scalar-load wait counter.  Rebuilding each pointer as a global one
// from its address lets the compiler use global accesses (the kernels' arrays are all in global
// memory).
template <class T>
__device__ __forceinline__ T *glb(T *p) {
    typedef __attribute__((address_space(1))) T gT;
    return (T *)(gT *)(uintptr_t)p;
}

struct One {
    Member m;
    int64_t ntiles;
    __device__ Member at(int) const { return m; }
    __device__ int find(int64_t) const { return 0; }
};

struct Many {
    const Member *ms;  // device table, ascending tile0
    int nm;
    int64_t ntiles;
    __device__ Member at(int i) const {
        Member m = ms[i];
        m.T = glb(m.T);
        m.q = glb(m.q);
        m.pm = glb(m.pm);
        m.pi = glb(m.pi);
        m.z = glb(m.z);
        m.phis = glb(m.phis);
        m.pblh = glb(m.pblh);
        m.tke = glb(m.tke);
        conv_deep_out_t &d = m.dout;
        d.dTdt = glb(d.dTdt);
        d.dqdt = glb(d.dqdt);
        d.mu = glb(d.mu);
        d.md = glb(d.md);
        d.prec = glb(d.prec);
        d.cape = glb(d.cape);
        d.klaunch = glb(d.klaunch);
        d.ktop = glb(d.ktop);
        d.trig = glb(d.trig);
        d.status = glb(d.status);
        conv_shallow_out_t &h = m.sout;
        h.dTdt = glb(h.dTdt);
        h.dqdt = glb(h.dqdt);
        h.mu = glb(h.mu);
        h.prec = glb(h.prec);
        h.cin = glb(h.cin);
        h.kbase = glb(h.kbase);
        h.ktop = glb(h.ktop);
        h.status = glb(h.status);
        return m;
    }
    // The member holding `tile`: the last entry with tile0 <= tile (members without columns share
    // their successor's tile0 and are skipped).
    __device__ int find(int64_t tile) const {
        int lo = 0, hi = nm - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) / 2;
            if (ms[mid].tile0 <= tile) lo = mid;
            else hi = mid - 1;
        }
        return lo;
    }
};

#define AT(arr, k) (arr)[(int64_t)(k) * ld + col]


// ------------------------------------------------------------------ wavefront compaction
// Appends the lanes with `pred` set to the list counted by *counter: one ballot, one popcount and
// one atomicAdd per wavefront.  Must be reached by every lane of the wavefront.
__device__ __forceinline__ int wave_append(bool pred, int *counter) {
    const unsigned long long m = __ballot(pred);
    if (m == 0ull) return -1;
    const int lane = __lane_id();
    const int leader = __ffsll((long long)m) - 1;
    int base = 0;
    if (lane == leader) base = atomicAdd(counter, (int)__popcll(m));
    base = __shfl(base, leader);
    return pred ? base + (int)__popcll(m & ((1ull << lane) - 1ull)) : -1;
}

// Launch shape: wavefronts per compute unit of the persistent deep-plume and shallow-plume
// passes (launched as one-wavefront blocks).
struct Launch {
    int fused_wpc, shallow_wpc;
};
constexpr int MAX_BPC = 8;               // 256-thread units per CU the workspace is sized for
constexpr int MAX_WPC = MAX_BPC * NWAVES;  // = 32 wavefronts per CU
constexpr Launch DEFAULT_LAUNCH = {5, 32};

struct Layout {
    size_t cnt, dlist, dmem, dkb, dkt, dkd, dcape, dSA, dSB;
    size_t slist, smem, sks, sflag, shs, sqs, scin, sMc, ssig2, members, dscr, sscr, total;
    int64_t threads;  // largest persistent grid (threads) the launch shape allows
    int lmax;
};

int device_cus();   // compute units of the current device (256 if it cannot be queried)
int check_launch();  // CONV_OK, or CONV_EHIP after recording the pending launch error

inline Member make_member(int64_t ncol, int nlev, const conv_params_t &P, const conv_state_t *s,
                   const conv_deep_out_t *d, const conv_shallow_out_t *sh, int64_t tile0) {
    Member m;
    memset(&m, 0, sizeof(m));
    m.T = s->T;
    m.q = s->q;
    m.pm = s->p_mid;
    m.pi = s->p_int;
    m.z = s->z;
    m.phis = s->phis;
    m.pblh = s->pblh;
    m.tke = s->tke;
    m.ld = s->ld;
    m.dt = s->dt;
    m.ncol = ncol;
    m.tile0 = tile0;
    m.nlev = nlev;
    m.P = P;
    if (d) m.dout = *d;
    if (sh) m.sout = *sh;
    return m;
}

}  // namespace cvk

constexpr int CONV_NSTAGES = 5;  // reset, trigger, deep plume, shallow re-trigger, shallow plume

struct conv_ctx {
    int64_t ncol;
    int nlev;
    conv_params_t P;
    char *ws;
    size_t ws_bytes;
    cvk::Layout lay;
    cvk::Launch launch;
    int cus;
    // Optional per-kernel timing: CONV_NSTAGES+1 events per recorded call.
    hipEvent_t *ev;
    int ev_cap, ev_used;
};

