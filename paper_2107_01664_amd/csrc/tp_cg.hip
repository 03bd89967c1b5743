// Persistent FP64 conjugate gradients for the Poisson solves of the preconditioner
// (Sec. 5.2: A~^{-1} = C^{-1} L^sigma C^{-1}, with C the cotan stiffness matrix).
//
// One cooperative launch solves k right-hand sides.  Columns are split into groups of KG;
// group g is served by the workgroups with blockIdx % ngroups == g, which partition the
// rows into contiguous chunks.  Workgroups of a group synchronise through a counter /
// generation barrier in global memory (agent-scope atomics), so the launch needs no host
// round trip per iteration.  Each iteration uses two barriers:
//   1. q = C p_new with p_new = r + beta p_old formed on the fly from the previous
//      iteration's r and p_old (p is double-buffered, so no workgroup overwrites values
//      another workgroup may still read), local p.q sums   -> barrier, alpha = r.r / p.q
//   2. x += alpha p_new, r -= alpha q, local r.r sums        -> barrier, beta, convergence
// Every workgroup adds the per-workgroup partial sums in the same order, so all of them
// take identical decisions and the result does not depend on scheduling.  Spins are
// bounded: a barrier that waits too long raises an abort flag and every workgroup exits.
#include "tp_internal.h"

namespace tp {

constexpr int kCgBlock = 256;
constexpr unsigned long long kSpinLimit = 1ull << 22;
constexpr int kBarStride = 64;      // unsigned words between the barriers of two groups

struct CgArgs {
    int64_t n;
    const int32_t* off;
    const int32_t* col;
    const double* val;
    const double* b;
    double* x;
    double* r;
    double* q;
    double* p;            // [2][n * k]
    double* red;          // [ngroups][2][W][KG]
    unsigned* bar;        // [ngroups][kBarStride]
    int* iters;
    double* relres;
    int* flags;
    double rtol;
    int maxiter;
    int k;
    int ngroups;
    int W;
};

__device__ bool group_barrier(unsigned* cnt, unsigned* gen, unsigned W, int* flags)
{
    __shared__ int ok_sh;
    __syncthreads();
    if (threadIdx.x == 0) {
        int ok = 1;
        __threadfence();
        const unsigned g = __hip_atomic_load(gen, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
        const unsigned prev = __hip_atomic_fetch_add(cnt, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        if (prev + 1 == W) {
            __hip_atomic_store(cnt, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(gen, g + 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            unsigned long long spins = 0;
            while (__hip_atomic_load(gen, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == g) {
                __builtin_amdgcn_s_sleep(1);
                ++spins;
                if (spins > kSpinLimit) {
                    ok = 0;
                    break;
                }
                if ((spins & 255ull) == 0ull &&
                    __hip_atomic_load(&flags[kFlagCgAbort], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                    ok = 0;
                    break;
                }
            }
            if (!ok) __hip_atomic_store(&flags[kFlagCgAbort], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        __threadfence();
        if (__hip_atomic_load(&flags[kFlagCgAbort], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) ok = 0;
        ok_sh = ok;
    }
    __syncthreads();
    return ok_sh != 0;
}

// Sum v over the workgroup for each of KG columns; result valid in sh_out[0..KG).
template <int KG>
__device__ __forceinline__ void block_sums(const double (&v)[KG], double* sh_wave, double* sh_out)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int c = 0; c < KG; ++c) {
        double s = v[c];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
        if (lane == 0) sh_wave[wave * KG + c] = s;
    }
    __syncthreads();
    if (threadIdx.x < KG) {
        double s = 0.0;
        for (int w = 0; w < kCgBlock / 64; ++w) s += sh_wave[w * KG + threadIdx.x];
        sh_out[threadIdx.x] = s;
    }
    __syncthreads();
}

template <int KG>
__global__ __launch_bounds__(kCgBlock) void k_cg(CgArgs A)
{
    __shared__ double sh_wave[(kCgBlock / 64) * KG];
    __shared__ double sh_sum[KG];
    __shared__ double sh_grp[KG];

    const int g = blockIdx.x % A.ngroups;
    const int w = blockIdx.x / A.ngroups;
    const int c0 = g * KG;
    const int nc = min(KG, A.k - c0);
    const int k = A.k;
    const int64_t chunk = (A.n + A.W - 1) / A.W;
    const int64_t rb = (int64_t)w * chunk, re = min(A.n, rb + chunk);
    unsigned* cnt = A.bar + (int64_t)g * kBarStride;
    unsigned* gen = cnt + kBarStride / 2;
    double* red0 = A.red + ((int64_t)g * 2 + 0) * A.W * KG;
    double* red1 = A.red + ((int64_t)g * 2 + 1) * A.W * KG;
    double* p0 = A.p;
    double* p1 = A.p + A.n * k;

    // Group-wide sum of the per-workgroup partials in workgroup order.
    auto group_sum = [&](double* red) {
        if (threadIdx.x < KG) {
            double s = 0.0;
            for (int ww = 0; ww < A.W; ++ww) s += red[ww * KG + threadIdx.x];
            sh_grp[threadIdx.x] = s;
        }
        __syncthreads();
    };

    double loc[KG];
#pragma unroll
    for (int c = 0; c < KG; ++c) loc[c] = 0.0;
    for (int64_t i = rb + threadIdx.x; i < re; i += kCgBlock) {
#pragma unroll
        for (int c = 0; c < KG; ++c) {
            if (c < nc) {
                const int64_t id = i * k + c0 + c;
                const double bv = A.b[id];
                A.x[id] = 0.0;
                A.r[id] = bv;
                p0[id] = 0.0;
                loc[c] += bv * bv;
            }
        }
    }
    block_sums<KG>(loc, sh_wave, sh_sum);
    if (threadIdx.x < KG) red0[w * KG + threadIdx.x] = sh_sum[threadIdx.x];
    if (!group_barrier(cnt, gen, (unsigned)A.W, A.flags)) return;
    group_sum(red0);

    double rr[KG], bb[KG], beta[KG], alpha[KG];
    bool done[KG];
    int its[KG];
#pragma unroll
    for (int c = 0; c < KG; ++c) {
        rr[c] = sh_grp[c];
        bb[c] = rr[c];
        beta[c] = 0.0;
        alpha[c] = 0.0;
        done[c] = (c >= nc) || !(bb[c] > 0.0);
        its[c] = 0;
    }
    __syncthreads();

    for (int it = 0; it < A.maxiter; ++it) {
        bool all = true;
#pragma unroll
        for (int c = 0; c < KG; ++c) all = all && done[c];
        if (all) break;
        double* pold = (it & 1) ? p1 : p0;
        double* pnew = (it & 1) ? p0 : p1;

        // 1. p_new = r + beta p_old (own rows); q = C p_new from the previous values.
#pragma unroll
        for (int c = 0; c < KG; ++c) loc[c] = 0.0;
        for (int64_t i = rb + threadIdx.x; i < re; i += kCgBlock) {
            double acc[KG];
#pragma unroll
            for (int c = 0; c < KG; ++c) acc[c] = 0.0;
            for (int32_t e = A.off[i]; e < A.off[i + 1]; ++e) {
                const int64_t jb = (int64_t)A.col[e] * k + c0;
                const double v = A.val[e];
#pragma unroll
                for (int c = 0; c < KG; ++c)
                    if (c < nc) acc[c] += v * (A.r[jb + c] + beta[c] * pold[jb + c]);
            }
#pragma unroll
            for (int c = 0; c < KG; ++c) {
                if (c < nc) {
                    const int64_t id = i * k + c0 + c;
                    const double pn = A.r[id] + beta[c] * pold[id];
                    pnew[id] = pn;
                    A.q[id] = acc[c];
                    loc[c] += pn * acc[c];
                }
            }
        }
        block_sums<KG>(loc, sh_wave, sh_sum);
        if (threadIdx.x < KG) red1[w * KG + threadIdx.x] = sh_sum[threadIdx.x];
        if (!group_barrier(cnt, gen, (unsigned)A.W, A.flags)) return;
        group_sum(red1);
#pragma unroll
        for (int c = 0; c < KG; ++c) alpha[c] = done[c] ? 0.0 : rr[c] / sh_grp[c];
        __syncthreads();

        // 2. x += alpha p_new, r -= alpha q.
#pragma unroll
        for (int c = 0; c < KG; ++c) loc[c] = 0.0;
        for (int64_t i = rb + threadIdx.x; i < re; i += kCgBlock) {
#pragma unroll
            for (int c = 0; c < KG; ++c) {
                if (c < nc) {
                    const int64_t id = i * k + c0 + c;
                    A.x[id] += alpha[c] * pnew[id];
                    const double rn = A.r[id] - alpha[c] * A.q[id];
                    A.r[id] = rn;
                    loc[c] += rn * rn;
                }
            }
        }
        block_sums<KG>(loc, sh_wave, sh_sum);
        if (threadIdx.x < KG) red0[w * KG + threadIdx.x] = sh_sum[threadIdx.x];
        if (!group_barrier(cnt, gen, (unsigned)A.W, A.flags)) return;
        group_sum(red0);
#pragma unroll
        for (int c = 0; c < KG; ++c) {
            if (!done[c]) {
                const double rn = sh_grp[c];
                its[c] = it + 1;
                beta[c] = rn / rr[c];
                rr[c] = rn;
                if (sqrt(rn / bb[c]) <= A.rtol) done[c] = true;
            }
        }
        __syncthreads();
    }
    if (w == 0 && threadIdx.x < nc) {
        const int c = threadIdx.x;
        A.iters[c0 + c] = its[c];
        A.relres[c0 + c] = bb[c] > 0.0 ? sqrt(rr[c] / bb[c]) : 0.0;
    }
}

namespace {

struct CgShape {
    int kg, ngroups, W;
};

CgShape cg_shape(int64_t n, int k)
{
    CgShape s;
    s.kg = (k + 7) / 8;                       // at most 8 groups
    if (s.kg > kMaxGroupCols) s.kg = kMaxGroupCols;
    s.ngroups = (k + s.kg - 1) / s.kg;
    int64_t W = (n + 2047) / 2048;
    if (W < 1) W = 1;
    if (W > 32) W = 32;
    s.W = (int)W;
    return s;
}

template <int KG>
hipError_t launch_cg_k(const CgArgs& a, hipStream_t s)
{
    const void* fn = (const void*)k_cg<KG>;
    int per_cu = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kCgBlock, 0);
    if (e != hipSuccess) return e;
    const int64_t total = (int64_t)a.ngroups * a.W;
    if (total > (int64_t)per_cu * device_info().num_cu) return hipErrorCooperativeLaunchTooLarge;
    CgArgs args = a;
    void* params[] = {&args};
    return hipLaunchCooperativeKernel(fn, dim3((unsigned)total), dim3(kCgBlock), params, 0, s);
}

}  // namespace

size_t cg_red_doubles(int k)
{
    return (size_t)8 * 2 * 32 * kMaxGroupCols + (size_t)k;
}

size_t cg_bar_words(int k)
{
    (void)k;
    return (size_t)8 * kBarStride;
}

hipError_t launch_cg(int64_t n, const int32_t* off, const int32_t* col, const double* val,
                     const double* b, double* x, int k, double rtol, int maxiter,
                     const CgWork& w, hipStream_t s)
{
    const CgShape sh = cg_shape(n, k);
    hipError_t e = hipMemsetAsync(w.bar, 0, cg_bar_words(k) * sizeof(unsigned), s);
    if (e != hipSuccess) return e;
    CgArgs a;
    a.n = n; a.off = off; a.col = col; a.val = val; a.b = b; a.x = x;
    a.r = w.r; a.q = w.q; a.p = w.p; a.red = w.red; a.bar = w.bar;
    a.iters = w.iters; a.relres = w.relres; a.flags = w.flags;
    a.rtol = rtol; a.maxiter = maxiter; a.k = k; a.ngroups = sh.ngroups; a.W = sh.W;
    switch (sh.kg) {
    case 1: return launch_cg_k<1>(a, s);
    case 2: return launch_cg_k<2>(a, s);
    case 3: return launch_cg_k<3>(a, s);
    case 4: return launch_cg_k<4>(a, s);
    case 5: return launch_cg_k<5>(a, s);
    case 6: return launch_cg_k<6>(a, s);
    case 7: return launch_cg_k<7>(a, s);
    case 8: return launch_cg_k<8>(a, s);
    case 9: return launch_cg_k<9>(a, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace tp
