// Declarations of the conjugate-gradient solvers and the device-side synchronisation of
// their persistent kernels, shared by tp_cg.hip, tp_pcg.hip and tp_api.hip (not part of
// the C-ABI).
#pragma once

#include "tp_internal.h"

namespace tp {

// Persistent FP64 conjugate gradients on k columns (row-major [n][k]) with the matrix in
// column-major ELL form.  x gets the solution of C x = b (b must be per-component mean
// zero); iteration counts and final relative residuals per column go to device arrays.
struct CgWork {
    double* Z = nullptr;        // cg_state_doubles(n, k)
    double* p = nullptr;        // n * k
    double* red = nullptr;      // cg_red_doubles(k)
    unsigned* bar = nullptr;    // cg_bar_words(k)
    int* iters = nullptr;       // k
    double* relres = nullptr;   // k
    int* flags = nullptr;       // device error flags
};
size_t cg_red_doubles(int k);
size_t cg_bar_words(int k);
size_t cg_state_doubles(int64_t n, int k);
hipError_t launch_csr_to_ell(int64_t n, const int32_t* off, const int32_t* col, const double* val,
                             int w, int32_t* ecol, double* eval, hipStream_t s);
hipError_t launch_cg(int64_t n, const int32_t* ecol, const double* eval, int ell_w,
                     const double* b, double* x, int k, double rtol, int maxiter,
                     const CgWork& w, hipStream_t s);

// Two-level additive Schwarz preconditioned CG (blocks of pcg_block_size() vertices in
// (component, Morton) order, dense block inverses in LDS; Galerkin coarse correction on
// aggregates of consecutive blocks with four coarse functions each: an orthonormal basis of
// {1, x, y, z} on the aggregate's vertices).
constexpr int kPcgRowSlots = 8;          // aggregates one row's entries reach, at most
constexpr int kPcgRegSlots = 4;          // of them, kept in registers by the solver
struct PcgSetup {
    int64_t n = 0;
    int nb = 0;
    int na = 0;                           // aggregates
    int nc = 0;                           // coarse functions (4 per aggregate)
    int ell_w = 0;
    const int32_t* perm = nullptr;        // [n] block order -> vertex
    const int32_t* pcol = nullptr;        // [ell_w][n] permuted ELL columns
    double* pval = nullptr;               // [ell_w][n] permuted ELL values (per geometry)
    const int32_t* bstart = nullptr;      // [nb + 1]
    const int32_t* whole = nullptr;       // [nb] block is a whole component
    const int32_t* blk = nullptr;         // [n] block of each (permuted) row
    const int32_t* astart = nullptr;      // [na + 1] first block of each aggregate
    const int32_t* agg_of_block = nullptr;// [nb]
    const int32_t* acomp = nullptr;       // [na] component of each aggregate
    const int32_t* abl_off = nullptr;     // [nb + 1] aggregates touching each block
    const int32_t* abl = nullptr;         //          (sorted, the block's own included)
    const int8_t* rslot = nullptr;        // [kPcgRowSlots][n] slots (in the block's list) of the
                                          // aggregates a row touches, -1 when unused
    const int8_t* eslot = nullptr;        // [ell_w][n] row slot of each ELL entry
    double* phi = nullptr;                // [n][4] coarse functions at each row (per geometry)
    double* rw = nullptr;                 // [kPcgRowSlots][4][n] sum over a row's entries of one
                                          // aggregate of C_ij phi_j (per geometry)
    double* esum = nullptr;               // [nc] sum of each coarse function (per geometry)
    float* Binv = nullptr;                // [nb][bs][bs], FP32
    double* C0inv = nullptr;              // [nc][nc] (the coarse matrix, then its inverse)
};
struct PcgWork {
    double* Vb = nullptr;       // 2 * n * k   (two copies, see the kernel)
    double* rho = nullptr;      // 2 * nb * k
    double* red = nullptr;      // 2 * nb * 3k
    unsigned* bar = nullptr;
    int* iters = nullptr;
    double* relres = nullptr;
    int* flags = nullptr;
};
int pcg_block_size();
int pcg_max_blocks();                    // blocks of one problem, at most
int pcg_max_coarse();                    // coarse functions of one problem, at most
int pcg_max_block_aggregates();          // aggregates touching one block, at most
// Per-geometry set-up: permuted matrix values, block inverses, coarse functions, the
// coarse matrix and its inverse.  V: vertices (n x 3, caller order).
hipError_t launch_pcg_setup(const PcgSetup& ps, const double* V, const int32_t* lap_off, const double* lap_val,
                            hipStream_t s);
hipError_t launch_permute_rows(int64_t n, int k, const int32_t* perm, int ld, int c0, const double* src,
                               double* dst, bool forward, hipStream_t s);
// One system of a multi-problem solve: b, x in block order, [n][k].
struct PcgItem {
    const PcgSetup* ps = nullptr;
    const double* b = nullptr;
    double* x = nullptr;
    PcgWork w;
    double rtol = 1e-10;
    int maxiter = 1;
    int warm = 0;             // 1: x holds the initial guess (tolerance still relative to |b|)
};
// Device table entries for n systems (tab_dev) and their pinned host staging (tab_host):
// the host staging must not be rewritten before the copy enqueued here has run.
size_t pcg_table_bytes(int n);
// Solve the n systems (k columns each, k <= kMaxGroupCols) in as few cooperative launches
// as fit on the device at once; each system's arithmetic is that of a launch of its own.
hipError_t launch_pcg_batch(const PcgItem* items, int n, int k, void* tab_dev, void* tab_host,
                            hipStream_t s);

// Multi-launch form of the same solve for problems of more than pcg_max_blocks() blocks
// (up to pcg_max_blocks_multi()): one kernel per phase of an iteration, the host reading
// a device stop flag every few iterations (so the call returns after the solve has ended).
// b, x in block order [n][k], k <= kMaxGroupCols; work arrays [n][k] (r, p, s, m, an, v),
// shares [nb][4][kMaxGroupCols], g [nc][kMaxGroupCols], part pcg_ml_part_doubles(n),
// state pcg_ml_state_bytes() on the device and in pinned host memory.
struct PcgMlWork {
    double* r = nullptr;
    double* p = nullptr;
    double* s = nullptr;
    double* m = nullptr;
    double* an = nullptr;
    double* v = nullptr;
    double* shares = nullptr;
    double* g = nullptr;
    double* part = nullptr;
    void* state = nullptr;
    void* state_host = nullptr;
};
int pcg_max_blocks_multi();
size_t pcg_ml_state_bytes();
size_t pcg_ml_part_doubles(int64_t n);
hipError_t launch_pcg_ml(const PcgSetup& ps, const double* b, double* x, int k, double rtol, int maxiter,
                         const PcgMlWork& w, int* iters, double* relres, hipStream_t s);

// ------------------------------------------------------------------ device-side sync

constexpr unsigned long long kSpinLimit = 1ull << 22;
constexpr int kLine = 32;            // unsigned words per 128-byte line
// barrier words of one group: one flag line per workgroup, at most kMaxBarrierW workgroups
constexpr int kMaxBarrierW = 256;
constexpr int kBarWordsPerGroup = kMaxBarrierW * kLine;

#if defined(__HIPCC__)
// Sum of a double over the 64 lanes of a wave in a fixed order, returned uniformly:
// DPP quad swaps, half-row and row mirrors give each 16-lane row its sum in every lane
// (each step adds the same two values in every lane of a pair, so all lanes agree), then
// the four row sums are read and added as (r0 + r1) + (r2 + r3).
template <int CTRL>
__device__ __forceinline__ double dpp_move(double v)
{
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double read_lane(double v, int lane)
{
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double wave_sum(double v)
{
    v = v + dpp_move<0xB1>(v);    // quad_perm [1,0,3,2]
    v = v + dpp_move<0x4E>(v);    // quad_perm [2,3,0,1]
    v = v + dpp_move<0x141>(v);   // row_half_mirror
    v = v + dpp_move<0x140>(v);   // row_mirror
    return (read_lane(v, 0) + read_lane(v, 16)) + (read_lane(v, 32) + read_lane(v, 48));
}

// Loads and stores of the data that workgroups of one launch exchange across a
// group_barrier_direct: agent-scope relaxed atomics are made coherent at the device level
// by the memory system itself (the store is written through the XCD's L2, the load misses
// it), so no L2 write-back or invalidate is needed to pass them between XCDs.
__device__ __forceinline__ void xstore(double* p, double v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double xload(const double* p)
{
    return __hip_atomic_load(const_cast<double*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Barrier among the W workgroups of a group, the target-th of the launch (1, 2, ...): every
// workgroup raises its own flag word (one 128-byte line each, zeroed before the launch) to
// target, then all its threads poll the W flags (a few each) until all have reached it.
// No atomic read-modify-write is involved, so arrivals do not serialise on a counter.
// The workgroup barrier alone does not wait for global stores (it only orders them for
// waves of the same CU): so every wave first waits until its own stores have been
// acknowledged (s_waitcnt vmcnt(0), immediate 0x0F70: expcnt and lgkmcnt at their maxima),
// and thread 0 raises the flag only after all waves have done so.
//   FENCED: plain loads and stores may cross the barrier.  The flag store is an agent-scope
//   release (the XCD's L2 is written back first) and an agent-scope acquire fence after
//   the wait makes the other workgroups' stores visible to the whole workgroup (the caches
//   it invalidates are shared by the workgroup's waves).
//   Direct: only xstore / xload data may cross the barrier; their stores are complete at the
//   device coherence point once acknowledged, so the flag is a relaxed store and no cache
//   is written back or invalidated (about half the latency; the workgroup's L2 contents
//   survive the barrier).
// Spins are bounded: a wait that exceeds kSpinLimit, or sees the abort flag, sets the abort
// flag and returns false in every workgroup.
template <bool FENCED>
__device__ __forceinline__ bool group_barrier_t(unsigned* gbar, int w, int W, int* flags, unsigned target)
{
    __shared__ int ok_sh;
    __builtin_amdgcn_s_waitcnt(0x0F70);
    __syncthreads();
    if (threadIdx.x == 0) {
        if (FENCED)
            __hip_atomic_store(gbar + (size_t)w * kLine, target, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        else
            __hip_atomic_store(gbar + (size_t)w * kLine, target, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        ok_sh = 1;
    }
    __syncthreads();
    bool bad = false;
    for (int q = threadIdx.x; q < W && !bad; q += blockDim.x) {
        unsigned long long spins = 0;
        while (__hip_atomic_load(gbar + (size_t)q * kLine, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
            __builtin_amdgcn_s_sleep(1);
            ++spins;
            if (spins > kSpinLimit ||
                ((spins & 255ull) == 0ull &&
                 __hip_atomic_load(&flags[kFlagCgAbort], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))) {
                bad = true;
                break;
            }
        }
    }
    if (bad) {
        __hip_atomic_store(&flags[kFlagCgAbort], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        ok_sh = 0;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        if (FENCED) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        if (__hip_atomic_load(&flags[kFlagCgAbort], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) ok_sh = 0;
    }
    __syncthreads();
    return ok_sh != 0;
}

__device__ __forceinline__ bool group_barrier(unsigned* gbar, int w, int W, int* flags, unsigned target)
{
    return group_barrier_t<true>(gbar, w, W, flags, target);
}
__device__ __forceinline__ bool group_barrier_direct(unsigned* gbar, int w, int W, int* flags, unsigned target)
{
    return group_barrier_t<false>(gbar, w, W, flags, target);
}

#endif

}  // namespace tp
