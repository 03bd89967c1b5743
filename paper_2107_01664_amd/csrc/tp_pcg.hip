// Two-level additive Schwarz preconditioned CG for the cotan Poisson solves (Sec. 5.2).
//
// Unknowns are reordered by (connected component, Morton code of the vertex position) and
// cut into blocks of at most kBS consecutive vertices, so every block is a compact patch
// of the surface.  The preconditioner is
//     M^{-1} r = sum_B R_B^T C_BB^{-1} R_B r  +  R_0^T C_0^+ R_0 r,
// with C_BB the block's rows and columns of C (exact dense inverse, FP64) and C_0 the
// Galerkin coarse matrix of the block indicator vectors (C_0[B][B'] = sum of the entries
// of C between B and B').  A block that is a whole component, and the coarse matrix, are
// singular on the per-component constants; they are made invertible by adding the rank-one
// term (d / m) 1 1^T per component (d a diagonal scale, m its size), which leaves the action
// on per-component mean-zero vectors equal to the pseudo-inverse.
//
// The solver is the Chronopoulos-Gear form of preconditioned CG: with u = M^{-1} r and
// w = C u, the sums gamma = (r,u) and delta = (w,u) give beta = gamma / gamma_old and
// alpha = gamma / (delta - beta gamma / alpha_old), and p = u + beta p, s = w + beta s (= C p),
// x += alpha p, r -= alpha s.  One workgroup of kBS threads owns one block (one row per
// thread) and keeps its C_BB^{-1} in LDS for the whole solve.  An iteration has two grid
// exchanges (two-level counter barrier, bounded spin).  In the first, every block publishes
// its block solve v = C_BB^{-1} r_B and the block sums of r (coarse right-hand side); after
// it, every block forms the coarse values of its own and neighbouring blocks, u = v + c(block)
// and C u from the neighbours' v.  In the second, the block partials of (r,u), (w,u) and
// (r,r) are added.  All partial sums are added in block order by every workgroup, so every
// workgroup takes the same decisions and the result does not depend on scheduling.  (The
// pipelined form, which folds the sums into the next exchange, lost convergence here:
// relative perturbations of 1e-15 per iteration in its auxiliary recurrences already cost
// 15 % more iterations and 1e-13 stalled it, while this form is unchanged up to 1e-13.)
// Every solve ends by checking the true residual b - C x and restarts from it when the
// recursively updated residual has drifted.
#include "tp_internal.h"

#include <algorithm>
#include <type_traits>
#include <utility>
#include <vector>

namespace tp {

constexpr int kBS = 128;            // vertices per block = row-owning threads of a solver workgroup
constexpr int kThreads = 2 * kBS;   // threads per solver workgroup: row owners + helpers
constexpr int kMaxNbn = 32;         // neighbouring blocks of a block (itself included)
constexpr int kMaxNbPcg = 256;      // blocks (one co-resident workgroup per block)
static_assert(kMaxNbPcg <= kMaxBarrierW, "one barrier flag per block");

// ---------------------------------------------------------------- per-geometry setup

// Permuted ELL values: row inew of the permuted matrix is row perm[inew] of C, entries in
// CSR order (the permuted column indices were built with the pattern).
__global__ void k_perm_ell_vals(int64_t n, int w, const int32_t* __restrict__ perm,
                                const int32_t* __restrict__ off, const double* __restrict__ val,
                                double* __restrict__ pval)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t old = perm[i];
    const int32_t b = off[old], len = off[old + 1] - b;
    for (int e = 0; e < w; ++e) pval[(int64_t)e * n + i] = e < len ? val[b + e] : 0.0;
}

// Dense inverse of each diagonal block (Gauss-Jordan in LDS; the block is symmetric
// positive definite, or made so by the rank-one term, so no pivoting is needed).
constexpr int kInvThreads = 256;
__global__ __launch_bounds__(kInvThreads) void k_block_inverse(int64_t n, int w, const int32_t* __restrict__ pcol,
                                                       const double* __restrict__ pval,
                                                       const int32_t* __restrict__ bstart,
                                                       const int32_t* __restrict__ whole,
                                                       float* __restrict__ Binv)
{
    extern __shared__ __align__(16) double A[];   // kBS x kBS, row-major
    __shared__ double fcol[kBS];
    const int B = blockIdx.x;
    const int32_t s0 = bstart[B], cnt = bstart[B + 1] - s0;
    for (int t = threadIdx.x; t < kBS * kBS; t += kInvThreads) A[t] = 0.0;
    __syncthreads();
    for (int t = threadIdx.x; t < kBS; t += kInvThreads) {
        if (t < cnt) {
            const int64_t i = s0 + t;
            for (int e = 0; e < w; ++e) {
                const int32_t j = pcol[(int64_t)e * n + i];
                if (j >= s0 && j < s0 + cnt) A[t * kBS + (j - s0)] += pval[(int64_t)e * n + i];
            }
        } else {
            A[t * kBS + t] = 1.0;             // padding rows: identity
        }
    }
    __syncthreads();
    if (whole[B]) {
        // rank-one term (d / cnt) 1 1^T on the block, d = mean diagonal
        __shared__ double dsum;
        if (threadIdx.x == 0) {
            double s = 0.0;
            for (int t = 0; t < cnt; ++t) s += A[t * kBS + t];
            dsum = s / cnt;
        }
        __syncthreads();
        const double add = dsum / cnt;
        for (int t = threadIdx.x; t < cnt * cnt; t += kInvThreads) A[(t / cnt) * kBS + (t % cnt)] += add;
        __syncthreads();
    }
    for (int k = 0; k < kBS; ++k) {
        const double p = 1.0 / A[k * kBS + k];
        __syncthreads();
        if (threadIdx.x < kBS) fcol[threadIdx.x] = A[threadIdx.x * kBS + k];   // column k before the update
        __syncthreads();
        if (threadIdx.x < kBS) A[k * kBS + threadIdx.x] = (threadIdx.x == k ? 1.0 : A[k * kBS + threadIdx.x]) * p;
        __syncthreads();
        // each thread updates kBS * kBS / kInvThreads entries of one column, all loads issued
        // together
        const int j = threadIdx.x & (kBS - 1);
        const double akj = A[k * kBS + j];
#pragma unroll 16
        for (int i = threadIdx.x / kBS; i < kBS; i += kInvThreads / kBS) {
            if (i != k) {
                const double base = (j == k) ? 0.0 : A[i * kBS + j];
                A[i * kBS + j] = base - fcol[i] * akj;
            }
        }
        __syncthreads();
    }
    // symmetrize (the elimination leaves rounding-level asymmetry) and round to FP32
    float* dst = Binv + (int64_t)B * kBS * kBS;
    for (int t = threadIdx.x; t < kBS * kBS; t += kInvThreads) {
        const int i = t / kBS, j = t - i * kBS;
        dst[t] = (float)(0.5 * (A[i * kBS + j] + A[j * kBS + i]));
    }
}

// Coarse matrix rows: C0[B][B'] = sum over rows of B of the entries in columns of B', and
// bdiag[B] = sum of the diagonal entries of C over the rows of B.  One workgroup per block;
// thread 0 adds in row order (deterministic).
__global__ __launch_bounds__(64) void k_coarse_rows(int64_t n, int w, int nb, const int32_t* __restrict__ pcol,
                                                    const double* __restrict__ pval,
                                                    const int32_t* __restrict__ bstart,
                                                    const int32_t* __restrict__ blk,
                                                    double* __restrict__ C0, double* __restrict__ bdiag)
{
    extern __shared__ __align__(16) double acc[];   // nb
    const int B = blockIdx.x;
    for (int t = threadIdx.x; t < nb; t += blockDim.x) acc[t] = 0.0;
    __syncthreads();
    if (threadIdx.x == 0) {
        double dg = 0.0;
        for (int64_t i = bstart[B]; i < bstart[B + 1]; ++i)
            for (int e = 0; e < w; ++e) {
                const int32_t j = pcol[(int64_t)e * n + i];
                const double a = pval[(int64_t)e * n + i];
                acc[blk[j]] += a;
                if (j == i) dg += a;      // padding entries point at i with value 0
            }
        bdiag[B] = dg;
    }
    __syncthreads();
    for (int t = threadIdx.x; t < nb; t += blockDim.x) C0[(int64_t)B * nb + t] = acc[t];
}

// Inverse of the nb x nb coarse matrix after adding the per-component rank-one terms.  The
// rank-one scale of a component of several blocks is the mean diagonal of the coarse matrix
// over such blocks; a component of one block has a zero coarse entry (C is singular on its
// constants), so it gets the block's own diagonal sum of C instead (any positive scale gives
// the same action on mean-zero vectors; this one keeps rounding errors of the block sums from
// being amplified).  The matrix is symmetric positive definite, so no pivoting is needed.
constexpr int kCoarseThreads = 1024;
constexpr int kCoarseSweepMax = 200;   // packed upper triangle: 200 x 201 / 2 doubles = 157 KB of LDS

__device__ __forceinline__ double coarse_entry(const double* __restrict__ G, int nb, int i, int j,
                                               const int32_t* __restrict__ bcomp,
                                               const int32_t* __restrict__ ncomp_blocks,
                                               const double* __restrict__ bdiag, double dmean)
{
    // the block sums of the two triangles may differ in the last bit: their mean is used
    double v = 0.5 * (G[(int64_t)i * nb + j] + G[(int64_t)j * nb + i]);
    if (bcomp[i] == bcomp[j]) {
        const int nc = ncomp_blocks[bcomp[i]];
        v += nc > 1 ? dmean / nc : bdiag[i];
    }
    return v;
}

__device__ double coarse_dmean(const double* __restrict__ G, int nb, const int32_t* __restrict__ bcomp,
                               const int32_t* __restrict__ ncomp_blocks)
{
    double s = 0.0;
    int cnt = 0;
    for (int i = 0; i < nb; ++i)
        if (ncomp_blocks[bcomp[i]] > 1) {
            s += G[(int64_t)i * nb + i];
            ++cnt;
        }
    return cnt > 0 ? s / cnt : 0.0;
}

// nb <= kCoarseSweepMax: symmetric sweeps in LDS on the packed upper triangle (row i holds
// columns i .. nb-1).  Sweeping pivot k with d = a_kk maps a_ij -> a_ij - a_ik a_kj / d
// (i, j != k), a_ik -> a_ik / d, a_kk -> -1 / d; after all pivots the matrix is -A^{-1}.
// Rows are spread over the waves, columns over the lanes.
__global__ __launch_bounds__(kCoarseThreads) void k_coarse_sweep(int nb, const int32_t* __restrict__ bcomp,
                                                                 const int32_t* __restrict__ ncomp_blocks,
                                                                 const double* __restrict__ bdiag,
                                                                 double* __restrict__ G)
{
    extern __shared__ __align__(16) double A[];
    __shared__ double fcol[kMaxNbPcg];
    __shared__ double dmean_sh;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    constexpr int kWaves = kCoarseThreads / 64;
    auto off = [&](int i) { return i * nb - (i * (i - 1)) / 2; };
    if (threadIdx.x == 0) dmean_sh = coarse_dmean(G, nb, bcomp, ncomp_blocks);
    __syncthreads();
    const double dmean = dmean_sh;
    for (int i = wave; i < nb; i += kWaves)
        for (int j = i + lane; j < nb; j += 64) A[off(i) + j - i] = coarse_entry(G, nb, i, j, bcomp, ncomp_blocks, bdiag, dmean);
    __syncthreads();
    for (int k = 0; k < nb; ++k) {
        const double d = A[off(k)];
        if ((int)threadIdx.x < nb) {
            const int i = threadIdx.x;
            fcol[i] = i <= k ? A[off(i) + k - i] : A[off(k) + i - k];
        }
        __syncthreads();
        const double invd = 1.0 / d;
        for (int i = wave; i < nb; i += kWaves) {
            const double fi = fcol[i];
            for (int j = i + lane; j < nb; j += 64) {
                const int idx = off(i) + j - i;
                double v;
                if (i == k && j == k) v = -invd;
                else if (i == k) v = fcol[j] * invd;
                else if (j == k) v = fi * invd;
                else v = A[idx] - fi * fcol[j] * invd;
                A[idx] = v;
            }
        }
        __syncthreads();
    }
    for (int i = wave; i < nb; i += kWaves)
        for (int j = i + lane; j < nb; j += 64) {
            const double v = -A[off(i) + j - i];
            G[(int64_t)i * nb + j] = v;
            G[(int64_t)j * nb + i] = v;
        }
}

// nb > kCoarseSweepMax: Gauss-Jordan elimination on the full matrix in global memory.
__global__ __launch_bounds__(kCoarseThreads) void k_coarse_inverse(int nb, const int32_t* __restrict__ bcomp,
                                                                   const int32_t* __restrict__ ncomp_blocks,
                                                                   const double* __restrict__ bdiag,
                                                                   double* __restrict__ G)
{
    __shared__ double fcol[kMaxNbPcg];
    __shared__ double dmean_sh;
    const int nn = nb * nb;
    if (threadIdx.x == 0) dmean_sh = coarse_dmean(G, nb, bcomp, ncomp_blocks);
    __syncthreads();
    const double dmean = dmean_sh;
    // symmetrised entries with the rank-one terms: the upper triangle first (each pair read
    // and written by one thread), then the diagonal and the mirrored lower triangle
    double* A = G;
    {
        for (int t = threadIdx.x; t < nn; t += kCoarseThreads) {
            const int i = t / nb, j = t - i * nb;
            if (i < j) A[t] = coarse_entry(G, nb, i, j, bcomp, ncomp_blocks, bdiag, dmean);
        }
        __threadfence_block();
        __syncthreads();
        for (int t = threadIdx.x; t < nn; t += kCoarseThreads) {
            const int i = t / nb, j = t - i * nb;
            if (i == j) A[t] += ncomp_blocks[bcomp[i]] > 1 ? dmean / ncomp_blocks[bcomp[i]] : bdiag[i];
            else if (i > j) A[t] = A[(int64_t)j * nb + i];
        }
        __threadfence_block();
        __syncthreads();
    }
    for (int k = 0; k < nb; ++k) {
        const double p = 1.0 / A[(int64_t)k * nb + k];
        __syncthreads();
        for (int j = threadIdx.x; j < nb; j += kCoarseThreads) fcol[j] = A[(int64_t)j * nb + k];
        __syncthreads();
        for (int j = threadIdx.x; j < nb; j += kCoarseThreads)
            A[(int64_t)k * nb + j] = (j == k ? 1.0 : A[(int64_t)k * nb + j]) * p;
        __threadfence_block();
        __syncthreads();
#pragma unroll 8
        for (int t = threadIdx.x; t < nn; t += kCoarseThreads) {
            const int i = t / nb, j = t - i * nb;
            if (i != k) {
                const double base = (j == k) ? 0.0 : A[t];
                A[t] = base - fcol[i] * A[(int64_t)k * nb + j];
            }
        }
        __threadfence_block();
        __syncthreads();
    }
}

// forward: dst[i][c] = src[perm[i]][c0 + c] (dst in block order, row stride k);
// backward: dst[perm[i]][c0 + c] = src[i][c].  ld is the row stride of the vertex-order side.
__global__ void k_permute_rows(int64_t n, int k, const int32_t* __restrict__ perm, int ld, int c0,
                               const double* __restrict__ src, double* __restrict__ dst, int forward)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * k) return;
    const int64_t i = t / k;
    const int c = (int)(t - i * k);
    if (forward) dst[i * k + c] = src[(int64_t)perm[i] * ld + c0 + c];
    else dst[(int64_t)perm[i] * ld + c0 + c] = src[i * k + c];
}

// ---------------------------------------------------------------- solver

struct PcgArgs {
    int64_t n;
    int nb;
    int ell_w;
    const int32_t* pcol;      // [ell_w][n]
    const double* pval;       // [ell_w][n]
    const uint8_t* pslot;     // [ell_w][n] slot of the column's block in the row block's list
    const int32_t* bstart;    // [nb + 1]
    const int32_t* badj_off;  // [nb + 1]
    const int32_t* badj;      // neighbour blocks (sorted, itself included)
    const float* Binv;        // [nb][kBS][kBS], FP32
    const double* C0inv;      // [nb][nb]
    const double* b;          // [n][k] (block order)
    double* x;                // [n][k]
    double* Vb;               // [2][n][k] block solves, copy = barrier count % 2
    double* rho;              // [2][nb][k] block sums of the preconditioned vector
    double* red;              // [2][nb][3k] block partial sums
    unsigned* bar;
    int* iters;
    double* relres;
    int* flags;
    double rtol;
    int maxiter;
    int k;
    int block0;               // first workgroup of this problem in its launch
};

constexpr int kCrowMax = 7680;      // doubles of cached coarse-inverse rows (60 KB)

template <int KG>
struct PcgShared {
    float Binv[kBS * kBS];
    double crow[kCrowMax];          // rows of C0inv of the neighbouring blocks
    double r[kBS * KG];
    double rho[kMaxNbPcg * KG];
    double c[kMaxNbn * KG];
    double wave[(kThreads / 64) * 3 * KG];
    double sums[3 * KG];
    double coef[2 * KG];            // alpha, beta of every column
    int live[KG];                   // column not yet converged
    double part[kThreads];
    int32_t nbl[kMaxNbn];
};

// Sum of n values p[0], p[stride], ... in a fixed order: four interleaved partial sums, so
// four loads are in flight at a time, added as (s0 + s1) + (s2 + s3).
__device__ __forceinline__ double sum_fixed(const double* __restrict__ p, int n, int64_t stride)
{
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    int i = 0;
    for (; i + 4 <= n; i += 4) {
        const double v0 = p[(int64_t)i * stride], v1 = p[(int64_t)(i + 1) * stride];
        const double v2 = p[(int64_t)(i + 2) * stride], v3 = p[(int64_t)(i + 3) * stride];
        a0 += v0;
        a1 += v1;
        a2 += v2;
        a3 += v3;
    }
    for (; i < n; ++i) a0 += p[(int64_t)i * stride];
    return (a0 + a1) + (a2 + a3);
}

// Dot product sum_i a[i] b[i * bstride] in the same fixed order.
__device__ __forceinline__ double dot_fixed(const double* __restrict__ a, const double* __restrict__ b, int n,
                                            int bstride)
{
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    int i = 0;
    for (; i + 4 <= n; i += 4) {
        a0 += a[i] * b[i * bstride];
        a1 += a[i + 1] * b[(i + 1) * bstride];
        a2 += a[i + 2] * b[(i + 2) * bstride];
        a3 += a[i + 3] * b[(i + 3) * bstride];
    }
    for (; i < n; ++i) a0 += a[i] * b[i * bstride];
    return (a0 + a1) + (a2 + a3);
}

// Fixed-order workgroup reduction of M values per thread (kThreads threads): butterfly
// within each wave, then the waves added in order.  Result in out[0 .. M).
template <int M>
__device__ __forceinline__ void wg_reduce(const double (&v)[M], double* wave_sh, double* out)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < M; ++q) {
        const double s = wave_sum(v[q]);
        if (lane == 0) wave_sh[wave * M + q] = s;
    }
    __syncthreads();
    if ((int)threadIdx.x < M) {
        double a = wave_sh[threadIdx.x];
#pragma unroll
        for (int w = 1; w < kThreads / 64; ++w) a += wave_sh[w * M + threadIdx.x];
        out[threadIdx.x] = a;
    }
    __syncthreads();
}

// One launch solves the systems of ntab independent problems: problem m owns workgroups
// [tab[m].block0, tab[m + 1].block0) and synchronises only among them (its own barrier
// words), so its iterates are those of a launch of its own.
template <int KG>
__global__ __launch_bounds__(kThreads) void k_pcg(const PcgArgs* __restrict__ tab, int ntab)
{
    extern __shared__ __align__(16) char smem_raw[];
    PcgShared<KG>& S = *reinterpret_cast<PcgShared<KG>*>(smem_raw);
    int pm = 0;
    for (int q = 1; q < ntab; ++q)
        if ((int)blockIdx.x >= tab[q].block0) pm = q;
    const PcgArgs A = tab[pm];
    const int B = (int)blockIdx.x - A.block0;
    const int nb = A.nb, k = A.k;
    const int64_t n = A.n;
    const int32_t s0 = A.bstart[B], cnt = A.bstart[B + 1] - s0;
    // threads t < kBS own row s0 + t of the block (when t < cnt); threads kBS .. kThreads
    // help with the block product, the coarse values and the cross-block sums
    const int t = threadIdx.x;
    const bool act = t < cnt;
    const int64_t i = s0 + t;

    {
        const float4* src = reinterpret_cast<const float4*>(A.Binv + (int64_t)B * kBS * kBS);
        float4* dst = reinterpret_cast<float4*>(S.Binv);
        for (int q = t; q < kBS * kBS / 4; q += kThreads) dst[q] = src[q];
    }
    const int nbo = A.badj_off[B], nbn = A.badj_off[B + 1] - nbo;
    for (int q = t; q < nbn; q += kThreads) S.nbl[q] = A.badj[nbo + q];
    __syncthreads();
    // rows of C0inv for the neighbouring blocks stay in LDS when they fit
    const bool crow_lds = (int64_t)nbn * nb <= kCrowMax;
    if (crow_lds)
        for (int q = t; q < nbn * nb; q += kThreads) S.crow[q] = A.C0inv[(int64_t)S.nbl[q / nb] * nb + (q % nb)];
    __syncthreads();
    int own_slot = 0;
    for (int q = 0; q < nbn; ++q)
        if (S.nbl[q] == B) own_slot = q;

    constexpr int kCache = 8;
    int32_t cj[kCache];
    double cv[kCache];
    int cs[kCache];
#pragma unroll
    for (int e = 0; e < kCache; ++e) {
        const bool in = act && e < A.ell_w;
        cj[e] = in ? A.pcol[(int64_t)e * n + i] : 0;
        cv[e] = in ? A.pval[(int64_t)e * n + i] : 0.0;
        cs[e] = in ? A.pslot[(int64_t)e * n + i] : 0;
    }
    // coarse part of a row of C M^{-1}: the row's entries added per neighbouring block (the
    // first entry of each block carries the block's weight, the others weight 0)
    double cw[kCache];
#pragma unroll
    for (int e = 0; e < kCache; ++e) {
        bool first = true;
#pragma unroll
        for (int f = 0; f < e; ++f) first = first && (cs[f] != cs[e] || f >= A.ell_w);
        double w = 0.0;
#pragma unroll
        for (int f = e; f < kCache; ++f) w += (cs[f] == cs[e] && f < A.ell_w) ? cv[f] : 0.0;
        cw[e] = (first && e < A.ell_w) ? w : 0.0;
    }

    // Exchange buffers come in two copies: data published before the b-th barrier goes to
    // copy b % 2 and is read between barriers b and b + 1; the copy is written again only
    // before barrier b + 2, when every reader has arrived at barrier b + 1.
    int nbar = 0;
    auto pub = [&]() { return nbar & 1; };
    auto got = [&]() { return (nbar - 1) & 1; };
    auto sync = [&]() -> bool {
        const bool ok = group_barrier(A.bar, B, nb, A.flags, (unsigned)nbar + 1u);
        ++nbar;
        return ok;
    };
    auto vbuf = [&](int c) { return A.Vb + (int64_t)c * n * k; };
    auto rhob = [&](int c) { return A.rho + (int64_t)c * nb * k; };
    auto redb = [&](int c) { return A.red + (int64_t)c * nb * 3 * k; };

    // M sums over the nb blocks of the copy c of the published partials ([nb][3][k], the
    // first M / KG groups): each value is cut into P parts of consecutive blocks, one per
    // thread (all loads in flight at once), then the parts are added in order.
    auto grid_sum = [&](auto mtag, int c) {
        constexpr int M = decltype(mtag)::value;
        const double* red = redb(c);
        constexpr int P = kThreads / M;
        const int chunk = (nb + P - 1) / P;
        const int q = t / P, part = t - q * P;
        if (q < M) {
            const int g = q / KG, cc = q - g * KG;
            double acc = 0.0;
            if (cc < k) {
                const int b0 = part * chunk, b1 = min(nb, b0 + chunk);
                if (b1 > b0) acc = sum_fixed(red + (int64_t)b0 * 3 * k + g * k + cc, b1 - b0, 3 * k);
            }
            S.part[q * P + part] = acc;
        }
        __syncthreads();
        if (t < M) S.sums[t] = sum_fixed(S.part + t * P, P, 1);
        __syncthreads();
    };

    double x[KG], r[KG], p[KG], s[KG];
    double m[KG], an[KG];

    // One exchange for the vector y (own rows): before the barrier, v = C_BB^{-1} y_B and the
    // block sums of y (coarse right-hand side) are published; after it, m = M^{-1} y and
    // an = C M^{-1} y at the own rows (m = v + c, with the coarse values c of the own and
    // neighbouring blocks).
    auto round = [&](const double (&y)[KG]) -> bool {
        const int cp = pub();
        if (t < kBS) {
#pragma unroll
            for (int c = 0; c < KG; ++c) S.r[t * KG + c] = (act && c < k) ? y[c] : 0.0;
        }
        __syncthreads();
        double v[KG];
#pragma unroll
        for (int c = 0; c < KG; ++c) v[c] = 0.0;
        // padding rows of the block hold y = 0 and an identity block in C_BB^{-1}, so the
        // product runs over all kBS rows with a fixed trip count.  Row tt's sum is split in
        // two halves of j (owner: j < kBS / 2, helper tt + kBS: the rest), added in that
        // order; chunks of CH rows: all LDS loads of a chunk are issued before its FMAs.
        const int tt = t & (kBS - 1), jbeg = (t / kBS) * (kBS / 2);
        constexpr int CH = KG <= 3 ? 8 : (KG <= 6 ? 4 : 2);
#pragma unroll 1
        for (int j0 = jbeg; j0 < jbeg + kBS / 2; j0 += CH) {
            float bj[CH];
            double yj[CH * KG];
#pragma unroll
            for (int q = 0; q < CH; ++q) bj[q] = S.Binv[(j0 + q) * kBS + tt];
#pragma unroll
            for (int q = 0; q < CH * KG; ++q) yj[q] = S.r[j0 * KG + q];
#pragma unroll
            for (int q = 0; q < CH; ++q)
#pragma unroll
                for (int c = 0; c < KG; ++c) v[c] += (double)bj[q] * yj[q * KG + c];
        }
        // the helpers' halves go through S.rho, which is free until the block sums arrive
        if (t >= kBS) {
#pragma unroll
            for (int c = 0; c < KG; ++c) S.rho[tt * KG + c] = v[c];
        }
        __syncthreads();
        if (t < kBS) {
#pragma unroll
            for (int c = 0; c < KG; ++c) v[c] += S.rho[t * KG + c];
        }
        double tmp[KG];
#pragma unroll
        for (int c = 0; c < KG; ++c) tmp[c] = (act && c < k) ? y[c] : 0.0;
        wg_reduce<KG>(tmp, S.wave, S.sums);
        if (act)
#pragma unroll
            for (int c = 0; c < KG; ++c)
                if (c < k) vbuf(cp)[i * k + c] = v[c];
        if (t < KG && t < k) rhob(cp)[(int64_t)B * k + t] = S.sums[t];
        if (!sync()) return false;
        const double* Vb = vbuf(cp);
        const double* rho = rhob(cp);
        // the neighbours' block solves are loaded now, so that their latency overlaps the
        // block sums' load and the coarse values
        double vnb[kCache][KG];
        if (act) {
#pragma unroll
            for (int e = 0; e < kCache; ++e)
#pragma unroll
                for (int c = 0; c < KG; ++c)
                    vnb[e][c] = (e < A.ell_w && c < k) ? Vb[(int64_t)cj[e] * k + c] : 0.0;
        }
        // block sums of every block: four loads in flight per thread
        for (int q0 = t; q0 < nb * KG; q0 += 4 * kThreads) {
            double vv[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int qq = q0 + u * kThreads, bb = qq / KG, c = qq - bb * KG;
                vv[u] = (qq < nb * KG && c < k) ? rho[(int64_t)bb * k + c] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < 4; ++u)
                if (q0 + u * kThreads < nb * KG) S.rho[q0 + u * kThreads] = vv[u];
        }
        __syncthreads();
        // coarse values c(sl) = sum_bb C0inv[nbl[sl]][bb] rho[bb] for the nbn x KG jobs: each
        // job's dot product is cut into P parts of consecutive blocks (one per thread)
        const int jobs = nbn * KG;
        for (int j0 = 0; j0 < jobs; j0 += kThreads) {
            const int nj = min(kThreads, jobs - j0);
            const int P = max(1, kThreads / nj);
            const int chunk = (nb + P - 1) / P;
            const int jl = t / P, part = t - jl * P;
            if (jl < nj) {
                const int job = j0 + jl, sl = job / KG, c = job - sl * KG;
                const double* row = crow_lds ? S.crow + sl * nb : A.C0inv + (int64_t)S.nbl[sl] * nb;
                const int b0 = part * chunk, b1 = min(nb, b0 + chunk);
                S.part[jl * P + part] = b1 > b0 ? dot_fixed(row + b0, S.rho + b0 * KG + c, b1 - b0, KG) : 0.0;
            }
            __syncthreads();
            if (t < nj) S.c[j0 + t] = sum_fixed(S.part + t * P, P, 1);
            __syncthreads();
        }
        double acc[KG];
#pragma unroll
        for (int c = 0; c < KG; ++c) {
            m[c] = v[c] + S.c[own_slot * KG + c];
            acc[c] = 0.0;
        }
        if (act) {
#pragma unroll
            for (int e = 0; e < kCache; ++e)
#pragma unroll
                for (int c = 0; c < KG; ++c) acc[c] += cv[e] * vnb[e][c];
#pragma unroll
            for (int e = 0; e < kCache; ++e)
                if (cw[e] != 0.0) {
#pragma unroll
                    for (int c = 0; c < KG; ++c) acc[c] += cw[e] * S.c[cs[e] * KG + c];
                }
            for (int e = kCache; e < A.ell_w; ++e) {
                const int32_t j = A.pcol[(int64_t)e * n + i];
                const double a = A.pval[(int64_t)e * n + i];
                const int sl = A.pslot[(int64_t)e * n + i];
#pragma unroll
                for (int c = 0; c < KG; ++c)
                    if (c < k) acc[c] += a * (Vb[(int64_t)j * k + c] + S.c[sl * KG + c]);
            }
        }
#pragma unroll
        for (int c = 0; c < KG; ++c) an[c] = acc[c];
        return true;
    };

    // Second exchange of an iteration: S.sums = (r,m), (an,m), (r,r) per column, each added
    // over the blocks in block order.
    auto dots = [&]() -> bool {
        double tmp[3 * KG];
#pragma unroll
        for (int c = 0; c < KG; ++c) {
            const bool on = act && c < k;
            tmp[c] = on ? r[c] * m[c] : 0.0;
            tmp[KG + c] = on ? an[c] * m[c] : 0.0;
            tmp[2 * KG + c] = on ? r[c] * r[c] : 0.0;
        }
        wg_reduce<3 * KG>(tmp, S.wave, S.sums);
        const int cp = pub();
        if (t < 3 * KG) {
            const int g = t / KG, c = t - g * KG;
            if (c < k) redb(cp)[(int64_t)B * 3 * k + g * k + c] = S.sums[t];
        }
        if (!sync()) return false;
        grid_sum(std::integral_constant<int, 3 * KG>{}, cp);
        return true;
    };

    // true residual r = b - C x; S.sums[0 .. KG) = |r|^2 per column
    auto true_residual = [&]() -> bool {
        if (act)
#pragma unroll
            for (int c = 0; c < KG; ++c)
                if (c < k) A.x[i * k + c] = x[c];
        if (!sync()) return false;
        double acc[KG];
#pragma unroll
        for (int c = 0; c < KG; ++c) acc[c] = 0.0;
        if (act) {
#pragma unroll
            for (int e = 0; e < kCache; ++e)
                if (e < A.ell_w)
#pragma unroll
                    for (int c = 0; c < KG; ++c)
                        if (c < k) acc[c] += cv[e] * A.x[(int64_t)cj[e] * k + c];
            for (int e = kCache; e < A.ell_w; ++e) {
                const int32_t j = A.pcol[(int64_t)e * n + i];
                const double a = A.pval[(int64_t)e * n + i];
#pragma unroll
                for (int c = 0; c < KG; ++c)
                    if (c < k) acc[c] += a * A.x[(int64_t)j * k + c];
            }
        }
        double tmp[KG];
#pragma unroll
        for (int c = 0; c < KG; ++c) {
            r[c] = (act && c < k) ? A.b[i * k + c] - acc[c] : 0.0;
            tmp[c] = r[c] * r[c];
        }
        wg_reduce<KG>(tmp, S.wave, S.sums);
        const int cp = pub();
        if (t < KG && t < k) redb(cp)[(int64_t)B * 3 * k + t] = S.sums[t];
        if (!sync()) return false;
        grid_sum(std::integral_constant<int, KG>{}, cp);
        return true;
    };

    // Thread c < KG keeps the scalars of column c (|b|^2, last |r|^2, gamma, alpha, state,
    // iterations) and forms its alpha and beta; the others read them from LDS.
    const double rtol2 = A.rtol * A.rtol;
    double my_bb = 0.0, my_rr = 0.0, my_gam = 0.0, my_alpha = 0.0;
    bool my_done = false;
    int my_its = 0;
#pragma unroll
    for (int c = 0; c < KG; ++c) {
        r[c] = (act && c < k) ? A.b[i * k + c] : 0.0;
        x[c] = 0.0;
    }
    int total_it = 0;
    constexpr int kMaxRestarts = 6;
    bool have_bb = false;
    for (int cycle = 0; cycle <= kMaxRestarts; ++cycle) {
        // ---- a cycle starts from the current (true) residual r
#pragma unroll
        for (int c = 0; c < KG; ++c) p[c] = s[c] = 0.0;
        bool first = true;
        for (;;) {
            if (!round(r)) return;           // m = M^{-1} r, an = C m
            if (!dots()) return;             // (r,m), (an,m), (r,r)
            const bool can = total_it < A.maxiter;
            if (t < KG) {
                const double g = S.sums[t], d = S.sums[KG + t];
                my_rr = S.sums[2 * KG + t];
                if (!have_bb) {
                    my_bb = my_rr;
                    my_done = (t >= k) || !(my_bb > 0.0);
                }
                double al = 0.0, be = 0.0;
                const bool live = !my_done && my_rr > rtol2 * my_bb;
                if (live) {
                    if (can) {
                        if (first) {
                            al = g / d;
                        } else {
                            be = g / my_gam;
                            al = g / (d - be * g / my_alpha);
                        }
                        my_its = total_it + 1;
                    }
                    my_gam = g;
                    my_alpha = al;
                }
                S.coef[t] = al;
                S.coef[KG + t] = be;
                S.live[t] = live ? 1 : 0;
            }
            have_bb = true;
            __syncthreads();
            bool conv = true;
#pragma unroll
            for (int c = 0; c < KG; ++c) {
                // columns that converged (or are done) have alpha = 0: x and r stay
                const double al = S.coef[c], be = S.coef[KG + c];
                conv = conv && S.live[c] == 0;
                p[c] = m[c] + be * p[c];
                s[c] = an[c] + be * s[c];
                x[c] += al * p[c];
                r[c] -= al * s[c];
            }
            if (conv || !can) break;
            ++total_it;
            first = false;
        }
        // ---- verify: recompute the true residual, restart from it if needed
        if (!true_residual()) return;
        if (t < KG) {
            if (!my_done) {
                my_rr = S.sums[t];
                if (my_rr <= rtol2 * my_bb) my_done = true;
            }
            S.live[t] = my_done ? 0 : 1;
        }
        __syncthreads();
        bool all = true;
#pragma unroll
        for (int c = 0; c < KG; ++c) all = all && S.live[c] == 0;
        __syncthreads();
        if (all || total_it >= A.maxiter) break;
    }
    if (act)
#pragma unroll
        for (int c = 0; c < KG; ++c)
            if (c < k) A.x[i * k + c] = x[c];
    if (B == 0 && t < k) {
        A.iters[t] = my_its;
        A.relres[t] = my_bb > 0.0 ? sqrt(my_rr / my_bb) : 0.0;
    }
}

// ---------------------------------------------------------------- launchers

size_t pcg_smem_bytes(int kg)
{
    switch (kg) {
    case 1: return sizeof(PcgShared<1>);
    case 2: return sizeof(PcgShared<2>);
    case 3: return sizeof(PcgShared<3>);
    case 4: return sizeof(PcgShared<4>);
    case 5: return sizeof(PcgShared<5>);
    case 6: return sizeof(PcgShared<6>);
    case 7: return sizeof(PcgShared<7>);
    case 8: return sizeof(PcgShared<8>);
    case 9: return sizeof(PcgShared<9>);
    default: return 0;
    }
}

hipError_t launch_pcg_setup(const PcgSetup& ps, const int32_t* lap_off, const double* lap_val,
                            hipStream_t s)
{
    hipLaunchKernelGGL(k_perm_ell_vals, dim3((unsigned)((ps.n + 255) / 256)), dim3(256), 0, s,
                       ps.n, ps.ell_w, ps.perm, lap_off, lap_val, ps.pval);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const size_t binv_smem = sizeof(double) * kBS * kBS;
    e = hipFuncSetAttribute((const void*)k_block_inverse, hipFuncAttributeMaxDynamicSharedMemorySize, (int)binv_smem);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_block_inverse, dim3(ps.nb), dim3(256), binv_smem, s, ps.n, ps.ell_w, ps.pcol,
                       ps.pval, ps.bstart, ps.whole, ps.Binv);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    double* bdiag = ps.C0inv + (int64_t)ps.nb * ps.nb;   // scratch tail of the C0inv buffer
    hipLaunchKernelGGL(k_coarse_rows, dim3(ps.nb), dim3(64), sizeof(double) * ps.nb, s, ps.n, ps.ell_w,
                       ps.nb, ps.pcol, ps.pval, ps.bstart, ps.blk, ps.C0inv, bdiag);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (ps.nb <= kCoarseSweepMax) {
        const size_t sm = sizeof(double) * (size_t)ps.nb * (ps.nb + 1) / 2;
        e = hipFuncSetAttribute((const void*)k_coarse_sweep, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)(sizeof(double) * kCoarseSweepMax * (kCoarseSweepMax + 1) / 2));
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_coarse_sweep, dim3(1), dim3(kCoarseThreads), sm, s, ps.nb, ps.bcomp,
                           ps.ncomp_blocks, bdiag, ps.C0inv);
    } else {
        hipLaunchKernelGGL(k_coarse_inverse, dim3(1), dim3(kCoarseThreads), 0, s, ps.nb, ps.bcomp,
                           ps.ncomp_blocks, bdiag, ps.C0inv);
    }
    return hipGetLastError();
}

hipError_t launch_permute_rows(int64_t n, int k, const int32_t* perm, int ld, int c0, const double* src,
                               double* dst, bool forward, hipStream_t s)
{
    hipLaunchKernelGGL(k_permute_rows, dim3((unsigned)((n * k + 255) / 256)), dim3(256), 0, s, n, k, perm,
                       ld, c0, src, dst, forward ? 1 : 0);
    return hipGetLastError();
}

namespace {

const void* pcg_fn(int k)
{
    switch (k) {
    case 1: return (const void*)k_pcg<1>;
    case 2: return (const void*)k_pcg<2>;
    case 3: return (const void*)k_pcg<3>;
    case 4: return (const void*)k_pcg<4>;
    case 5: return (const void*)k_pcg<5>;
    case 6: return (const void*)k_pcg<6>;
    case 7: return (const void*)k_pcg<7>;
    case 8: return (const void*)k_pcg<8>;
    case 9: return (const void*)k_pcg<9>;
    default: return nullptr;
    }
}

}  // namespace

bool pcg_supported(int64_t nb, int ncomp_blocks_max) { (void)ncomp_blocks_max; return nb >= 1 && nb <= kMaxNbPcg; }
int pcg_block_size() { return kBS; }
int pcg_max_neighbors() { return kMaxNbn; }
size_t pcg_table_bytes(int n) { return sizeof(PcgArgs) * (size_t)std::max(n, 1); }

hipError_t launch_pcg_batch(const PcgItem* items, int n, int k, void* tab_dev, void* tab_host,
                            hipStream_t s)
{
    if (n < 1) return hipSuccess;
    const void* fn = pcg_fn(k);
    if (!fn) return hipErrorInvalidValue;
    const size_t smem = pcg_smem_bytes(k);
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
    if (e != hipSuccess) return e;
    int per_cu = 0;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kThreads, smem);
    if (e != hipSuccess) return e;
    const int64_t cap = (int64_t)per_cu * device_info().num_cu;
    PcgArgs* H = static_cast<PcgArgs*>(tab_host);
    for (int m = 0; m < n; ++m) {
        const PcgItem& it = items[m];
        const PcgSetup& ps = *it.ps;
        PcgArgs& a = H[m];
        a.n = ps.n; a.nb = ps.nb; a.ell_w = ps.ell_w; a.pcol = ps.pcol; a.pval = ps.pval; a.pslot = ps.pslot;
        a.bstart = ps.bstart; a.badj_off = ps.badj_off; a.badj = ps.badj; a.Binv = ps.Binv; a.C0inv = ps.C0inv;
        a.b = it.b; a.x = it.x; a.Vb = it.w.Vb; a.rho = it.w.rho; a.red = it.w.red; a.bar = it.w.bar;
        a.iters = it.w.iters; a.relres = it.w.relres; a.flags = it.w.flags;
        a.rtol = it.rtol; a.maxiter = it.maxiter; a.k = k; a.block0 = 0;
        if ((int64_t)ps.nb > cap) return hipErrorCooperativeLaunchTooLarge;
    }
    // launches of consecutive problems whose workgroups are resident together
    std::vector<std::pair<int, int>> groups;
    for (int i0 = 0; i0 < n;) {
        int64_t sum = 0;
        int i1 = i0;
        while (i1 < n && sum + H[i1].nb <= cap) {
            H[i1].block0 = (int)sum;
            sum += H[i1].nb;
            ++i1;
        }
        groups.emplace_back(i0, i1);
        i0 = i1;
    }
    e = hipMemcpyAsync(tab_dev, tab_host, sizeof(PcgArgs) * n, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return e;
    for (int m = 0; m < n; ++m) {
        e = hipMemsetAsync(items[m].w.bar, 0, kBarWordsPerGroup * sizeof(unsigned), s);
        if (e != hipSuccess) return e;
    }
    for (const auto& g : groups) {
        const PcgArgs* t = static_cast<const PcgArgs*>(tab_dev) + g.first;
        int nt = g.second - g.first;
        int blocks = 0;
        for (int m = g.first; m < g.second; ++m) blocks += H[m].nb;
        void* params[] = {(void*)&t, (void*)&nt};
        e = hipLaunchCooperativeKernel(fn, dim3(blocks), dim3(kThreads), params, smem, s);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace tp
