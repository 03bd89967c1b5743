// Two-level additive Schwarz preconditioned CG for the cotan Poisson solves (Sec. 5.2).
//
// Unknowns are reordered by (connected component, Morton code of the vertex position on
// the component's bounding cube) and cut into blocks of at most kBS consecutive vertices,
// so every block is a compact patch of the surface.  The preconditioner is
//     M^{-1} r = sum_B R_B^T C_BB^{-1} R_B r  +  Phi C_0^{-1} Phi^T r,
// with C_BB the block's rows and columns of C (dense inverse by register-tiled
// Gauss-Jordan, stored in FP32) and Phi a linear coarse space: aggregates of consecutive
// blocks of one component, each carrying an orthonormalised basis of {1, x, y, z} centred
// and scaled on the aggregate.  C_0 = Phi^T C Phi is assembled from per-row coarse weights;
// per component the rank-one term d e e^T / (e^T e) (e the coefficients of the component's
// constant, d the mean kept diagonal) makes it definite and leaves its action on
// per-component mean-zero vectors equal to the pseudo-inverse.
//
// The solver is the Chronopoulos-Gear form of preconditioned CG: with u = M^{-1} r and
// w = C u, the sums gamma = (r,u) and delta = (w,u) give beta = gamma / gamma_old and
// alpha = gamma / (delta - beta gamma / alpha_old), and p = u + beta p, s = w + beta s (= C p),
// x += alpha p, r -= alpha s.  One workgroup of 2 kBS threads owns one block (kBS row
// owners and kBS helpers for the block product) and keeps C_BB^{-1} for the whole solve: in
// LDS, or with four or more columns in registers, half a column per thread.  An iteration
// has two grid exchanges through per-workgroup flag lines, the
// exchanged values written and read as agent-scope atomics.  In the first, every block
// publishes its block solve v = C_BB^{-1} r_B and its shares Phi_B^T r of the coarse
// right-hand side; after it, every workgroup forms the coarse values of the aggregates its
// rows touch, u = v + Phi c and C u from the neighbours' v.  In the second, the block
// partials of (r,u), (w,u) and (r,r) are added.  All partial sums are added in block order
// by every workgroup, so every workgroup takes the same decisions and the result does not
// depend on scheduling.  (The pipelined form, which folds the sums into the next exchange,
// lost convergence here: relative perturbations of 1e-15 per iteration in its auxiliary
// recurrences already cost 15 % more iterations and 1e-13 stalled it, while this form is
// unchanged up to 1e-13.)  A solve may start from a given x (warm start; the tolerance
// stays relative to |b|).  Every solve ends by checking the true residual b - C x and
// restarts from it when the recursively updated residual has drifted.  Problems with more
// blocks than can be resident at once run the same iteration as one launch per phase
// (k_ml_*, further below).
#include "tp_solver.h"

#include <algorithm>
#include <type_traits>
#include <utility>
#include <vector>

namespace tp {

constexpr int kBS = 128;            // vertices per block = row-owning threads of a solver workgroup
constexpr int kThreads = 2 * kBS;   // threads per solver workgroup: row owners + helpers
constexpr int kMaxAggNbn = 16;      // aggregates touching a block (its own included)
constexpr int kMaxNbPcg = 256;      // blocks (one co-resident workgroup per block)
static_assert(kMaxNbPcg <= kMaxBarrierW, "one barrier flag per block");
constexpr int kMaxAggBlocks = 7;    // blocks per aggregate: ceil(4 kMaxNbPcg / kCoarseMax)
constexpr int kMaxNbMulti = 16384;  // blocks of the multi-launch solve (2,097,152 vertices)

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
// In-place Gauss-Jordan inverse of an n x n symmetric positive definite matrix (no
// pivoting) held in registers.  The matrix is NC x NC (NC = RB * NRB = CB * NCB; rows and
// columns n .. NC-1 zero); thread t < NRB * NCB holds the RB x CB tile a[r][c] =
// A[rb RB + r][cb CB + c] with rb = t % NRB, cb = t / NRB.  Pivot k with d = a_kk and
// g_i = a_ik / d:
//   a_ij -> a_ij - g_i a_kj (i, j != k),  a_kj -> a_kj / d,  a_ik -> -g_i,  a_kk -> 1 / d;
// row k takes the same multiply-add as the others with the multiplier 1 - 1/d.  Per pivot
// the pivot row and column pass through LDS (two copies, alternating, so one workgroup
// barrier per pivot suffices: a copy is written again only two pivots later, after every
// thread has passed the barrier in between); a thread reads CB + RB of their values for
// its RB CB multiply-adds.  The pivot's position within a tile is a compile-time constant
// of the unrolled inner loop (its length L is a multiple of RB and CB), so the tile stays
// in registers.  Threads t >= NRB * NCB only join the barriers.
template <int RB, int CB, int NRB, int NCB>
__device__ __forceinline__ void gj_inverse_tiles(double (&a)[RB][CB], int n, double* prow, double* fcol)
{
    constexpr int NC = RB * NRB;
    static_assert(CB * NCB == NC, "square tiling");
    constexpr int L = RB * CB / (RB % CB == 0 ? CB : (CB % RB == 0 ? RB : 1));   // RB, CB | L
    static_assert(L % RB == 0 && L % CB == 0, "unrolled pivots cover whole tiles");
    const int t = threadIdx.x;
    const bool on = t < NRB * NCB;
    const int rb = t % NRB, cb = t / NRB;
    int buf = 0;
    for (int k0 = 0; k0 < n; k0 += L) {
#pragma unroll
        for (int kk = 0; kk < L; ++kk) {
            const int k = k0 + kk;
            if (k < n) {
                const int rk = kk % RB, ck = kk % CB;   // position of row / column k in a tile
                double* pr = prow + buf * NC;
                double* fc = fcol + buf * NC;
                if (on && rb == k / RB) {
#pragma unroll
                    for (int c = 0; c < CB; ++c) pr[cb * CB + c] = a[rk][c];
                }
                if (on && cb == k / CB) {
#pragma unroll
                    for (int r = 0; r < RB; ++r) fc[rb * RB + r] = a[r][ck];
                }
                __syncthreads();
                const double invd = 1.0 / pr[k];
                if (on) {
                    double p[CB], g[RB], h[RB];
#pragma unroll
                    for (int c = 0; c < CB; ++c) p[c] = pr[cb * CB + c];
#pragma unroll
                    for (int r = 0; r < RB; ++r) {
                        g[r] = fc[rb * RB + r] * invd;
                        h[r] = rb * RB + r == k ? 1.0 - invd : g[r];
                    }
#pragma unroll
                    for (int r = 0; r < RB; ++r)
#pragma unroll
                        for (int c = 0; c < CB; ++c) a[r][c] = __builtin_fma(-h[r], p[c], a[r][c]);
                    if (cb == k / CB) {
#pragma unroll
                        for (int r = 0; r < RB; ++r) a[r][ck] = rb * RB + r == k ? invd : -g[r];
                    }
                }
                buf ^= 1;
            }
        }
    }
}

// Inverse of block B by one workgroup of kInvThreads threads.
constexpr int kInvThreads = 512;
__device__ __forceinline__ void block_inverse(int B, int64_t n, int w, const int32_t* __restrict__ pcol,
                                              const double* __restrict__ pval, const int32_t* __restrict__ bstart,
                                              const int32_t* __restrict__ whole, float* __restrict__ Binv)
{
    extern __shared__ __align__(16) double A[];   // kBS x kBS, row-major
    __shared__ double prow[2 * kBS], fcol[2 * kBS];
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
    // tiles of 4 rows x 8 columns: 32 row blocks x 16 column blocks
    constexpr int RB = 4, CB = 8, NRB = kBS / RB, NCB = kBS / CB;
    static_assert(NRB * NCB == kInvThreads, "one tile per thread");
    const int rb = threadIdx.x % NRB, cb = threadIdx.x / NRB;
    double a[RB][CB];
#pragma unroll
    for (int r = 0; r < RB; ++r)
#pragma unroll
        for (int c = 0; c < CB; ++c) a[r][c] = A[(rb * RB + r) * kBS + cb * CB + c];
    gj_inverse_tiles<RB, CB, NRB, NCB>(a, kBS, prow, fcol);
    __syncthreads();
#pragma unroll
    for (int r = 0; r < RB; ++r)
#pragma unroll
        for (int c = 0; c < CB; ++c) A[(rb * RB + r) * kBS + cb * CB + c] = a[r][c];
    __syncthreads();
    // symmetrize (the elimination leaves rounding-level asymmetry) and round to FP32
    float* dst = Binv + (int64_t)B * kBS * kBS;
    for (int t = threadIdx.x; t < kBS * kBS; t += kInvThreads) {
        const int i = t / kBS, j = t - i * kBS;
        dst[t] = (float)(0.5 * (A[i * kBS + j] + A[j * kBS + i]));
    }
}

// ---- coarse space: per aggregate, an orthonormal basis (in the Euclidean product on the
// aggregate's vertices) of {1, x, y, z}, with x, y, z centred and scaled on the aggregate.
// It is the Cholesky factor L of the 4 x 4 Gram matrix that orthonormalises: phi = V L^-T.
// A function whose remainder after the previous ones is below 1e-6 of its norm (a flat or
// tiny aggregate) is dropped: its values are zero and its coarse row and column are zero
// but for a unit diagonal.

constexpr int kAggThreads = 256;

// Fixed-order sum of M values per thread over a kAggThreads workgroup.
template <int M>
__device__ __forceinline__ void agg_sum(const double (&v)[M], double* sh, double* out)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < M; ++q) {
        const double s = wave_sum(v[q]);
        if (lane == 0) sh[wave * M + q] = s;
    }
    __syncthreads();
    if ((int)threadIdx.x < M) {
        double a = 0.0;
        for (int w = 0; w < kAggThreads / 64; ++w) a += sh[w * M + threadIdx.x];
        out[threadIdx.x] = a;
    }
    __syncthreads();
}

// One workgroup per aggregate: phi[i][0..4) for its rows (block order) and esum[4g + a].
__global__ __launch_bounds__(kAggThreads) void k_agg_basis(const int32_t* __restrict__ perm,
                                                             const double* __restrict__ V,
                                                             const int32_t* __restrict__ astart,
                                                             const int32_t* __restrict__ bstart,
                                                             double* __restrict__ phi, double* __restrict__ esum)
{
    __shared__ double sh[(kAggThreads / 64) * 10];
    __shared__ double tot[10];
    __shared__ double T[16];
    const int g = blockIdx.x;
    const int v0 = bstart[astart[g]], v1 = bstart[astart[g + 1]];
    const double m = (double)(v1 - v0);
    // centroid
    double ps[3] = {0.0, 0.0, 0.0};
    for (int i = v0 + (int)threadIdx.x; i < v1; i += kAggThreads) {
        const int64_t o = (int64_t)perm[i] * 3;
        ps[0] += V[o]; ps[1] += V[o + 1]; ps[2] += V[o + 2];
    }
    agg_sum<3>(ps, sh, tot);
    const double cx = tot[0] / m, cy = tot[1] / m, cz = tot[2] / m;
    __syncthreads();
    // scale: largest coordinate offset (a maximum does not depend on the order)
    double pm[1] = {0.0};
    for (int i = v0 + (int)threadIdx.x; i < v1; i += kAggThreads) {
        const int64_t o = (int64_t)perm[i] * 3;
        pm[0] = fmax(pm[0], fmax(fabs(V[o] - cx), fmax(fabs(V[o + 1] - cy), fabs(V[o + 2] - cz))));
    }
    {
        const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
        double w = pm[0];
        for (int off = 32; off > 0; off >>= 1) w = fmax(w, __shfl_xor(w, off));
        if (lane == 0) sh[wave] = w;
        __syncthreads();
        if (threadIdx.x == 0) {
            double a = 0.0;
            for (int q = 0; q < kAggThreads / 64; ++q) a = fmax(a, sh[q]);
            tot[0] = a > 0.0 ? 1.0 / a : 1.0;
        }
        __syncthreads();
    }
    const double is = tot[0];
    __syncthreads();
    // Gram matrix of (1, x', y', z'): entries (0,0) (0,1) (0,2) (0,3) (1,1) (1,2) (1,3) (2,2) (2,3) (3,3)
    double gs[10];
#pragma unroll
    for (int q = 0; q < 10; ++q) gs[q] = 0.0;
    for (int i = v0 + (int)threadIdx.x; i < v1; i += kAggThreads) {
        const int64_t o = (int64_t)perm[i] * 3;
        const double f[4] = {1.0, (V[o] - cx) * is, (V[o + 1] - cy) * is, (V[o + 2] - cz) * is};
        int q = 0;
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = a; b < 4; ++b) gs[q++] += f[a] * f[b];
    }
    agg_sum<10>(gs, sh, tot);
    if (threadIdx.x == 0) {
        double G[4][4];
        int q = 0;
        for (int a = 0; a < 4; ++a)
            for (int b = a; b < 4; ++b) G[a][b] = G[b][a] = tot[q++];
        // Cholesky with dropped pivots, then T = L^{-1} (rows of dropped functions zero)
        double L[4][4] = {};
        bool keep[4];
        for (int a = 0; a < 4; ++a) {
            double d = G[a][a];
            for (int c = 0; c < a; ++c) d -= L[a][c] * L[a][c];
            keep[a] = d > 1e-12 * G[a][a] && G[a][a] > 0.0;
            const double la = keep[a] ? sqrt(d) : 0.0;
            L[a][a] = la;
            for (int b = a + 1; b < 4; ++b) {
                double v = G[b][a];
                for (int c = 0; c < a; ++c) v -= L[b][c] * L[a][c];
                L[b][a] = keep[a] ? v / la : 0.0;
            }
        }
        double Ti[4][4] = {};
        for (int a = 0; a < 4; ++a) {
            if (!keep[a]) continue;
            Ti[a][a] = 1.0 / L[a][a];
            for (int b = 0; b < a; ++b) {
                double v = 0.0;
                for (int c = b; c < a; ++c) v += L[a][c] * Ti[c][b];
                Ti[a][b] = -v / L[a][a];
            }
        }
        for (int a = 0; a < 4; ++a)
            for (int b = 0; b < 4; ++b) T[a * 4 + b] = Ti[a][b];
    }
    __syncthreads();
    double es[4] = {0.0, 0.0, 0.0, 0.0};
    for (int i = v0 + (int)threadIdx.x; i < v1; i += kAggThreads) {
        const int64_t o = (int64_t)perm[i] * 3;
        const double f[4] = {1.0, (V[o] - cx) * is, (V[o + 1] - cy) * is, (V[o + 2] - cz) * is};
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            double v = 0.0;
#pragma unroll
            for (int b = 0; b < 4; ++b) v += T[a * 4 + b] * f[b];
            phi[(int64_t)i * 4 + a] = v;
            es[a] += v;
        }
    }
    agg_sum<4>(es, sh, tot);
    if (threadIdx.x < 4) esum[4 * g + threadIdx.x] = tot[threadIdx.x];
}

// Per row i and slot q (an aggregate the row's entries reach): rw[q][a][i] = sum over the
// entries j of that aggregate of C_ij phi_j[a], added in ELL order.
__global__ void k_row_coarse(int64_t n, int w, const int32_t* __restrict__ pcol, const double* __restrict__ pval,
                             const int8_t* __restrict__ eslot, const double* __restrict__ phi, double* __restrict__ rw)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double acc[kPcgRowSlots][4];
#pragma unroll
    for (int q = 0; q < kPcgRowSlots; ++q)
#pragma unroll
        for (int a = 0; a < 4; ++a) acc[q][a] = 0.0;
    for (int e = 0; e < w; ++e) {
        const int32_t j = pcol[(int64_t)e * n + i];
        const double c = pval[(int64_t)e * n + i];
        const int q = eslot[(int64_t)e * n + i];
#pragma unroll
        for (int qq = 0; qq < kPcgRowSlots; ++qq)
            if (qq == q)
#pragma unroll
                for (int a = 0; a < 4; ++a) acc[qq][a] += c * phi[(int64_t)j * 4 + a];
    }
#pragma unroll
    for (int q = 0; q < kPcgRowSlots; ++q)
#pragma unroll
        for (int a = 0; a < 4; ++a) rw[((int64_t)q * 4 + a) * n + i] = acc[q][a];
}

// Galerkin coarse matrix rows of aggregate g: C0[4g + a][4h + b] = sum over rows i of g of
// phi_i[a] rw[q(h)][b][i].  kAggThreads threads = 16 row groups x 16 (a, b) pairs; each group
// adds a contiguous share of the rows, the groups are added in order.
constexpr int kAsmGroups = kAggThreads / 16;
__global__ __launch_bounds__(kAggThreads) void k_coarse_assemble(int64_t n, int na, int nc,
                                                                   const int32_t* __restrict__ astart,
                                                                   const int32_t* __restrict__ bstart,
                                                                   const int32_t* __restrict__ blk,
                                                                   const int32_t* __restrict__ abl_off,
                                                                   const int32_t* __restrict__ abl,
                                                                   const int8_t* __restrict__ rslot,
                                                                   const double* __restrict__ phi,
                                                                   const double* __restrict__ rw,
                                                                   double* __restrict__ C0)
{
    extern __shared__ __align__(16) double acc[];   // [kAsmGroups][na][16]
    const int g = blockIdx.x;
    const int v0 = bstart[astart[g]], v1 = bstart[astart[g + 1]];
    for (int t = threadIdx.x; t < kAsmGroups * na * 16; t += kAggThreads) acc[t] = 0.0;
    __syncthreads();
    const int grp = threadIdx.x / 16, ab = threadIdx.x % 16, a = ab / 4, b = ab % 4;
    const int rows = v1 - v0, chunk = (rows + kAsmGroups - 1) / kAsmGroups;
    const int r0 = v0 + grp * chunk, r1 = min(v1, r0 + chunk);
    double* my = acc + (int64_t)grp * na * 16;
    for (int i = r0; i < r1; ++i) {
        const int B = blk[i];
        const double pa = phi[(int64_t)i * 4 + a];
#pragma unroll
        for (int q = 0; q < kPcgRowSlots; ++q) {
            const int sl = rslot[(int64_t)q * n + i];
            if (sl < 0) continue;
            const int h = abl[abl_off[B] + sl];
            my[h * 16 + ab] += pa * rw[((int64_t)q * 4 + b) * n + i];
        }
    }
    __syncthreads();
    for (int t = threadIdx.x; t < na * 16; t += kAggThreads) {
        double v = 0.0;
        for (int q = 0; q < kAsmGroups; ++q) v += acc[(int64_t)q * na * 16 + t];
        const int h = t / 16, aa = (t % 16) / 4, bb = t % 4;
        C0[(int64_t)(4 * g + aa) * nc + 4 * h + bb] = v;
    }
}

// Inverse of the nc x nc coarse matrix (nc <= kCoarseMax) after the regularisation of each
// component's constants: with e the coefficients of the component's constant function in the
// coarse basis (e_d = sum of coarse function d), the term dmean e e^T / (e^T e) is added,
// dmean the mean of the kept diagonal entries; the action on per-component mean-zero vectors
// is that of the pseudo-inverse.  The matrix is symmetric positive definite, so no pivoting
// is needed.
constexpr int kCoarseThreads = 512;
constexpr int kCoarseMax = 160;
// tiles of 5 rows x 10 columns: 32 row blocks x 16 column blocks
constexpr int kCoarseRB = 5, kCoarseCB = 10;
constexpr int kCoarseNRB = kCoarseMax / kCoarseRB, kCoarseNCB = kCoarseMax / kCoarseCB;
static_assert(kCoarseNRB * kCoarseNCB <= kCoarseThreads, "one tile per thread");
constexpr int kMaxCoarseComp = kCoarseMax / 4;
static_assert(kMaxAggBlocks * kCoarseMax >= 4 * kMaxNbPcg, "aggregates of up to kMaxAggBlocks blocks");

// One workgroup: the regularised matrix is formed in registers (a tile per thread),
// inverted there (gj_inverse_tiles) and written over G, each entry pair (i, j), (j, i)
// from the upper triangle, so the result is exactly symmetric.
__device__ __forceinline__ void coarse_inverse(int nc, const int32_t* __restrict__ acomp,
                                               const double* __restrict__ esum, double* __restrict__ G)
{
    __shared__ double prow[2 * kCoarseMax], fcol[2 * kCoarseMax];
    __shared__ double diag[kCoarseMax], es[kCoarseMax];
    __shared__ int32_t comp[kCoarseMax];
    __shared__ double enorm[kMaxCoarseComp];   // e^T e per component
    __shared__ double dmean_sh;
    const int t = threadIdx.x;
    if (t < nc) {
        diag[t] = G[(int64_t)t * nc + t];
        es[t] = esum[t];
        comp[t] = acomp[t / 4];   // components are numbered densely over the aggregates
    }
    __syncthreads();
    if (t == 0) {
        double sd = 0.0;
        int cnt = 0;
        for (int i = 0; i < nc; ++i)
            if (diag[i] > 0.0) {
                sd += diag[i];
                ++cnt;
            }
        dmean_sh = cnt > 0 ? sd / cnt : 1.0;
    }
    if (t < kMaxCoarseComp) {
        double en = 0.0;
        for (int i = 0; i < nc; ++i)
            if (comp[i] == t) en += es[i] * es[i];
        enorm[t] = en;
    }
    __syncthreads();
    const double dmean = dmean_sh;
    constexpr int RB = kCoarseRB, CB = kCoarseCB, NRB = kCoarseNRB, NCB = kCoarseNCB;
    const bool on = t < NRB * NCB;
    const int rb = t % NRB, cb = t / NRB;
    double a[RB][CB];
#pragma unroll
    for (int r = 0; r < RB; ++r)
#pragma unroll
        for (int c = 0; c < CB; ++c) {
            const int i = rb * RB + r, j = cb * CB + c;
            double v = 0.0;
            if (on && i < nc && j < nc) {
                // the two triangles are assembled by different aggregates: their mean is used
                v = 0.5 * (G[(int64_t)i * nc + j] + G[(int64_t)j * nc + i]);
                const int ci = comp[i];
                if (ci == comp[j] && enorm[ci] > 0.0) v += dmean * es[i] * es[j] / enorm[ci];
                if (i == j && !(diag[i] > 0.0)) v = 1.0;   // dropped coarse function
            }
            a[r][c] = v;
        }
    // every thread has read its entries of G before the first barrier of the inversion, and
    // G is written only after the last one
    gj_inverse_tiles<RB, CB, NRB, NCB>(a, nc, prow, fcol);
#pragma unroll
    for (int r = 0; r < RB; ++r)
#pragma unroll
        for (int c = 0; c < CB; ++c) {
            const int i = rb * RB + r, j = cb * CB + c;
            if (on && i < nc && j < nc && j >= i) {
                G[(int64_t)i * nc + j] = a[r][c];
                G[(int64_t)j * nc + i] = a[r][c];
            }
        }
}

// The block inverses (workgroups 0 .. nb-1) and the coarse inverse (workgroup nb) in one
// launch: they are independent, so the coarse inverse's single workgroup runs beside the
// blocks' workgroups instead of after them.
static_assert(kCoarseThreads == kInvThreads, "one workgroup size for both inverses");
__global__ __launch_bounds__(kInvThreads) void k_inverses(int nb, int64_t n, int w, const int32_t* __restrict__ pcol,
                                                          const double* __restrict__ pval,
                                                          const int32_t* __restrict__ bstart,
                                                          const int32_t* __restrict__ whole, float* __restrict__ Binv,
                                                          int nc, const int32_t* __restrict__ acomp,
                                                          const double* __restrict__ esum, double* __restrict__ G)
{
    if ((int)blockIdx.x < nb) block_inverse((int)blockIdx.x, n, w, pcol, pval, bstart, whole, Binv);
    else coarse_inverse(nc, acomp, esum, G);
}

__global__ void k_fill_zero(double* __restrict__ p, int64_t n)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) p[t] = 0.0;
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
    int nc;                   // coarse functions (4 per aggregate)
    int ell_w;
    const int32_t* pcol;      // [ell_w][n]
    const double* pval;       // [ell_w][n]
    const int32_t* bstart;    // [nb + 1]
    const int32_t* astart;    // [na + 1] first block of each aggregate
    const int32_t* agg_of_block;
    const int32_t* abl_off;   // [nb + 1] aggregates touching each block (sorted, own included)
    const int32_t* abl;
    const int8_t* rslot;      // [kPcgRowSlots][n], filled in order, -1 after the last
    const double* phi;        // [n][4]
    const double* rw;         // [kPcgRowSlots][4][n]
    const float* Binv;        // [nb][kBS][kBS], FP32
    const double* C0inv;      // [nc][nc]
    const double* b;          // [n][k] (block order)
    double* x;                // [n][k]
    double* Vb;               // [2][n][k] block solves, copy = barrier count % 2
    double* rho;              // [2][nb][4][k] block sums of phi times the preconditioned vector
    double* red;              // [2][nb][3k] block partial sums
    unsigned* bar;
    int* iters;
    double* relres;
    int* flags;
    double rtol;
    int maxiter;
    int k;
    int block0;               // first workgroup of this problem in its launch
    int stage;                // the block shares fit the LDS staging area after PcgShared
    int warm;                 // 1: x holds an initial guess (the previous solution)
};

constexpr int kCrowMax = 7680;      // cached coarse-inverse entries (FP32: 30 KB)

// With four or more columns a thread keeps its half column of the block inverse in
// registers; with fewer the inverse stays in LDS (the same product, bit for bit: measured on
// the 40,000-face torus, registers took 5 % off a 9-column solve, 3 % off a 6-column one,
// and were no faster with 3).
template <int KG>
constexpr bool kRegInv = KG >= 4;

template <int KG>
struct PcgShared {
    alignas(16) float Binv[kRegInv<KG> ? 4 : kBS * kBS];
    alignas(16) float crow[kCrowMax];   // rows of C0inv of the coarse functions of the touching
                                        // aggregates, rounded to FP32 (as the block inverses are)
    alignas(16) float r[kBS * KG];      // the vector of the block product, rounded to FP32
                                        // (16-byte aligned: read four values at a time)
    double rho[kCoarseMax * KG];    // coarse right-hand side [nc][KG] (and the block product's halves)
    double c[kMaxAggNbn * 4 * KG];  // coarse values [slot][4][KG]
    double wave[(kThreads / 64) * 4 * KG];
    double sums[4 * KG];
    double coef[2 * KG];            // alpha, beta of every column
    int live[KG];                   // column not yet converged
    double part[kThreads];
    int32_t nbl[kMaxAggNbn];
    int32_t ast[kCoarseMax / 4 + 1];  // first block of each aggregate
};
static_assert(kCoarseMax >= kBS, "the block product's halves go through PcgShared::rho");

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

// Sum in a fixed order of n values published by other workgroups (loaded with xload):
// the loads of 8 values at a time are all in flight before they are added, value i to
// partial sum i % 4, and the partial sums are added as (s0 + s1) + (s2 + s3).
__device__ __forceinline__ double sum_fixed_x(const double* __restrict__ p, int n, int64_t stride)
{
    double a[4] = {0.0, 0.0, 0.0, 0.0};
    for (int i = 0; i < n; i += 8) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = i + u < n ? xload(p + (int64_t)(i + u) * stride) : 0.0;
#pragma unroll
        for (int u = 0; u < 8; ++u) a[u & 3] += v[u];
    }
    return (a[0] + a[1]) + (a[2] + a[3]);
}

// Dot product sum_i a[i] b[i * bstride] in a fixed order: the loads of 8 terms at a time
// are issued before they are added, term i to partial sum i % 4, and the partial sums are
// added as (s0 + s1) + (s2 + s3).
template <class TA, bool ROUND32 = false>
__device__ __forceinline__ double dot_fixed(const TA* __restrict__ a, const double* __restrict__ b, int n,
                                            int bstride)
{
    // the terms a[i] b[i], with a[i] rounded to FP32 first when ROUND32
    auto av = [&](int i) -> double { return ROUND32 ? (double)(float)a[i] : (double)a[i]; };
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    int i = 0;
    for (; i + 8 <= n; i += 8) {
        double x[8], y[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            x[u] = av(i + u);
            y[u] = b[(i + u) * bstride];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) acc[u & 3] += x[u] * y[u];
    }
    for (; i < n; ++i) acc[i & 3] += av(i) * b[i * bstride];
    return (acc[0] + acc[1]) + (acc[2] + acc[3]);
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
    // staging area for all blocks' coarse shares ([nb][4][k]), when the launch has room
    double* stg = reinterpret_cast<double*>(smem_raw + (sizeof(PcgShared<KG>) + 15) / 16 * 16);
    int pm = 0;
    for (int q = 1; q < ntab; ++q)
        if ((int)blockIdx.x >= tab[q].block0) pm = q;
    const PcgArgs A = tab[pm];
    const int B = (int)blockIdx.x - A.block0;
    const int nb = A.nb, nc = A.nc, k = A.k;
    const int64_t n = A.n;
    const int32_t s0 = A.bstart[B], cnt = A.bstart[B + 1] - s0;
    // threads t < kBS own row s0 + t of the block (when t < cnt); threads kBS .. kThreads
    // help with the block product, the coarse values and the cross-block sums
    const int t = threadIdx.x;
    const bool act = t < cnt;
    const int64_t i = s0 + t;

    // Thread t takes half of column tt of C_BB^{-1}: rows jbeg .. jbeg + kBS / 2 (the inverse
    // is symmetric, so these are row tt's entries), in registers or in LDS for the solve.
    const int tt = t & (kBS - 1), jbeg = (t / kBS) * (kBS / 2);
    float binv[kRegInv<KG> ? kBS / 2 : 1];
    if constexpr (kRegInv<KG>) {
        const float* src = A.Binv + (int64_t)B * kBS * kBS + tt;
#pragma unroll
        for (int q = 0; q < kBS / 2; ++q) binv[q] = src[(int64_t)(jbeg + q) * kBS];
    } else {
        const float4* src = reinterpret_cast<const float4*>(A.Binv + (int64_t)B * kBS * kBS);
        float4* dst = reinterpret_cast<float4*>(S.Binv);
        for (int q = t; q < kBS * kBS / 4; q += kThreads) dst[q] = src[q];
    }
    // aggregates touching this block (slots), and the rows of C0inv of their coarse functions
    const int nbo = A.abl_off[B], nsl = A.abl_off[B + 1] - nbo;
    for (int q = t; q < nsl; q += kThreads) S.nbl[q] = A.abl[nbo + q];
    for (int q = t; q <= nc / 4; q += kThreads) S.ast[q] = A.astart[q];
    __syncthreads();
    const bool crow_lds = (int64_t)nsl * 4 * nc <= kCrowMax;
    if (crow_lds)
        for (int q = t; q < nsl * 4 * nc; q += kThreads) {
            const int row = q / nc;   // slot * 4 + function
            S.crow[q] = (float)A.C0inv[(int64_t)(4 * S.nbl[row / 4] + row % 4) * nc + (q % nc)];
        }
    __syncthreads();
    int own_slot = 0;
    {
        const int own = A.agg_of_block[B];
        for (int q = 0; q < nsl; ++q)
            if (S.nbl[q] == own) own_slot = q;
    }

    constexpr int kCache = 8;
    int32_t cj[kCache];
    double cv[kCache];
#pragma unroll
    for (int e = 0; e < kCache; ++e) {
        const bool in = act && e < A.ell_w;
        cj[e] = in ? A.pcol[(int64_t)e * n + i] : 0;
        cv[e] = in ? A.pval[(int64_t)e * n + i] : 0.0;
    }
    // the row's coarse functions and, per touched aggregate, the coarse part of its row of C
    // (slots beyond kPcgRegSlots, rare, are read from memory when used)
    double phi[4], rwt[kPcgRegSlots][4];
    int rsl[kPcgRegSlots];
    int nq_row = 0;
    if (act)
        for (int q = 0; q < kPcgRowSlots; ++q) nq_row += A.rslot[(int64_t)q * n + i] >= 0 ? 1 : 0;
#pragma unroll
    for (int a = 0; a < 4; ++a) phi[a] = act ? A.phi[i * 4 + a] : 0.0;
#pragma unroll
    for (int q = 0; q < kPcgRegSlots; ++q) {
        rsl[q] = act ? (int)A.rslot[(int64_t)q * n + i] : -1;
#pragma unroll
        for (int a = 0; a < 4; ++a) rwt[q][a] = (rsl[q] >= 0) ? A.rw[((int64_t)q * 4 + a) * n + i] : 0.0;
    }

    // Exchange buffers come in two copies: data published before the b-th barrier goes to
    // copy b % 2 and is read between barriers b and b + 1; the copy is written again only
    // before barrier b + 2, when every reader has arrived at barrier b + 1.
    int nbar = 0;
    auto pub = [&]() { return nbar & 1; };
    auto got = [&]() { return (nbar - 1) & 1; };
    auto sync = [&]() -> bool {
        const bool ok = group_barrier_direct(A.bar, B, nb, A.flags, (unsigned)nbar + 1u);
        ++nbar;
        return ok;
    };
    auto vbuf = [&](int c) { return A.Vb + (int64_t)c * n * k; };
    auto rhob = [&](int c) { return A.rho + (int64_t)c * nb * 4 * k; };
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
                if (b1 > b0) acc = sum_fixed_x(red + (int64_t)b0 * 3 * k + g * k + cc, b1 - b0, 3 * k);
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
            for (int c = 0; c < KG; ++c) S.r[t * KG + c] = (act && c < k) ? (float)y[c] : 0.0f;
        }
        __syncthreads();
        // The block solve is a preconditioner: C_BB^{-1} (FP32) times y rounded to FP32, with
        // FP32 sums (the solution's accuracy comes from the FP64 residuals; the CG iteration
        // counts equal those of an FP64 product).  Padding rows of the block hold y = 0 and an
        // identity block in C_BB^{-1}, so the product runs over all kBS rows with a fixed trip
        // count.  Row tt's sum is split in two halves of j (owner: j < kBS / 2, helper
        // tt + kBS: the rest), added in that order; chunks of CH rows: all LDS loads of a chunk
        // are issued before its multiply-adds.
        float v32[KG];
#pragma unroll
        for (int c = 0; c < KG; ++c) v32[c] = 0.0f;
        if constexpr (kRegInv<KG>) {
            constexpr int CH = KG <= 6 ? 8 : 4;
#pragma unroll
            for (int q0 = 0; q0 < kBS / 2; q0 += CH) {
                float yj[CH * KG];
#pragma unroll
                for (int q = 0; q < CH * KG; ++q) yj[q] = S.r[(jbeg + q0) * KG + q];
#pragma unroll
                for (int q = 0; q < CH; ++q)
#pragma unroll
                    for (int c = 0; c < KG; ++c) v32[c] = __builtin_fmaf(binv[q0 + q], yj[q * KG + c], v32[c]);
            }
        } else {
            constexpr int CH = 8;
#pragma unroll 1
            for (int j0 = jbeg; j0 < jbeg + kBS / 2; j0 += CH) {
                float bj[CH], yj[CH * KG];
#pragma unroll
                for (int q = 0; q < CH; ++q) bj[q] = S.Binv[(j0 + q) * kBS + tt];
#pragma unroll
                for (int q = 0; q < CH * KG; ++q) yj[q] = S.r[j0 * KG + q];
#pragma unroll
                for (int q = 0; q < CH; ++q)
#pragma unroll
                    for (int c = 0; c < KG; ++c) v32[c] = __builtin_fmaf(bj[q], yj[q * KG + c], v32[c]);
            }
        }
        // the helpers' halves go through S.rho, which is free until the block sums arrive
        if (t >= kBS) {
#pragma unroll
            for (int c = 0; c < KG; ++c) S.rho[tt * KG + c] = (double)v32[c];
        }
        __syncthreads();
        double v[KG];
#pragma unroll
        for (int c = 0; c < KG; ++c) v[c] = t < kBS ? (double)v32[c] + S.rho[t * KG + c] : 0.0;
        // the block's share of the coarse right-hand side: sum over its rows of phi[a] y
        double tmp[4 * KG];
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int c = 0; c < KG; ++c) tmp[a * KG + c] = (act && c < k) ? phi[a] * y[c] : 0.0;
        wg_reduce<4 * KG>(tmp, S.wave, S.sums);
        if (act)
#pragma unroll
            for (int c = 0; c < KG; ++c)
                if (c < k) xstore(vbuf(cp) + i * k + c, v[c]);
        if (t < 4 * KG) {
            const int a = t / KG, c = t - a * KG;
            if (c < k) xstore(rhob(cp) + ((int64_t)B * 4 + a) * k + c, S.sums[t]);
        }
        if (!sync()) return false;
        const double* Vb = vbuf(cp);
        const double* rho = rhob(cp);
        // the neighbours' block solves: for up to 5 columns loaded now, so that their latency
        // overlaps the block sums' load and the coarse values; with more, after the block
        // sums (their kCache x KG loads would otherwise hold up the block sums' loads, which
        // return in order behind them), overlapping the coarse values
        double vnb[kCache][KG];
        auto load_vnb = [&]() {
            if (act) {
#pragma unroll
                for (int e = 0; e < kCache; ++e)
#pragma unroll
                    for (int c = 0; c < KG; ++c)
                        vnb[e][c] = (e < A.ell_w && c < k) ? xload(Vb + (int64_t)cj[e] * k + c) : 0.0;
            }
        };
        constexpr bool kVnbEarly = KG <= 5;
        if (kVnbEarly) load_vnb();
        if (A.stage) {
            // all blocks' shares in one contiguous, coalesced pass into LDS, then function
            // 4g + a of the coarse right-hand side sums aggregate g's blocks in block order
            // (the same sums, in the same order, as below)
            const int tot = nb * 4 * k;
            for (int e0 = t; e0 < tot; e0 += 8 * kThreads) {   // 8 loads in flight per thread
                double u8[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) u8[u] = e0 + u * kThreads < tot ? xload(rho + e0 + u * kThreads) : 0.0;
#pragma unroll
                for (int u = 0; u < 8; ++u)
                    if (e0 + u * kThreads < tot) stg[e0 + u * kThreads] = u8[u];
            }
            __syncthreads();
            for (int q = t; q < nc * KG; q += kThreads) {
                const int d = q / KG, c = q - d * KG, g = d / 4, a = d - 4 * g;
                double acc = 0.0;
                if (c < k)
                    for (int bb = S.ast[g]; bb < S.ast[g + 1]; ++bb) acc += stg[(bb * 4 + a) * k + c];
                S.rho[q] = acc;
            }
            __syncthreads();
        } else {
        // coarse right-hand side [nc][KG]: function 4g + a sums the shares of aggregate g's
        // blocks in block order.  Jobs q = t + jj kThreads of this thread: the loads of kJB
        // jobs (all of them for up to 3 columns; 2 at a time for more, to bound the registers
        // held) are issued before any is added.  An aggregate holds at most kMaxAggBlocks
        // blocks (the host never forms larger ones; any further blocks are added afterwards).
        constexpr int kJ = (kCoarseMax * KG + kThreads - 1) / kThreads;
        constexpr int kJB = KG <= 3 ? kJ : 2;
#pragma unroll 1
        for (int j0 = 0; j0 < kJ; j0 += kJB) {
            double sh[kJB][kMaxAggBlocks];
#pragma unroll
            for (int jj = 0; jj < kJB; ++jj) {
                const int q = t + (j0 + jj) * kThreads;
                const int d = q / KG, c = q - d * KG, g = d / 4, a = d - 4 * g;
                const bool on = q < nc * KG && c < k;
                const int b0 = on ? S.ast[g] : 0, cntb = on ? S.ast[g + 1] - b0 : 0;
#pragma unroll
                for (int u = 0; u < kMaxAggBlocks; ++u)
                    sh[jj][u] = u < cntb ? xload(rho + ((int64_t)(b0 + u) * 4 + a) * k + c) : 0.0;
            }
#pragma unroll
            for (int jj = 0; jj < kJB; ++jj) {
                const int q = t + (j0 + jj) * kThreads;
                if (q < nc * KG) {
                    const int d = q / KG, c = q - d * KG, g = d / 4, a = d - 4 * g;
                    double acc = 0.0;
#pragma unroll
                    for (int u = 0; u < kMaxAggBlocks; ++u) acc += sh[jj][u];
                    if (c < k)
                        for (int bb = S.ast[g] + kMaxAggBlocks; bb < S.ast[g + 1]; ++bb)
                            acc += xload(rho + ((int64_t)bb * 4 + a) * k + c);
                    S.rho[q] = acc;
                }
            }
        }
        __syncthreads();
        }
        if (!kVnbEarly) load_vnb();
        // coarse values S.c[sl][a][c] = sum_d C0inv[4 nbl[sl] + a][d] rho[d][c] for the
        // nsl x 4 x KG jobs: each job's dot product is cut into P parts (one per thread)
        const int jobs = nsl * 4 * KG;
        for (int j0 = 0; j0 < jobs; j0 += kThreads) {
            const int nj = min(kThreads, jobs - j0);
            const int P = max(1, kThreads / nj);
            const int chunk = (nc + P - 1) / P;
            const int jl = t / P, part = t - jl * P;
            if (jl < nj) {
                const int job = j0 + jl, row = job / KG, c = job - row * KG;   // row = slot * 4 + a
                const int d0 = part * chunk, d1 = min(nc, d0 + chunk);
                double pv = 0.0;
                if (d1 > d0) {
                    // the coarse-inverse entries in FP32 either way (the same operator for
                    // every block, whether its rows are cached in LDS or read from memory)
                    if (crow_lds)
                        pv = dot_fixed(S.crow + (int64_t)row * nc + d0, S.rho + d0 * KG + c, d1 - d0, KG);
                    else
                        pv = dot_fixed<double, true>(A.C0inv + (int64_t)(4 * S.nbl[row / 4] + row % 4) * nc + d0,
                                                     S.rho + d0 * KG + c, d1 - d0, KG);
                }
                S.part[jl * P + part] = pv;
            }
            __syncthreads();
            if (t < nj) S.c[j0 + t] = sum_fixed(S.part + t * P, P, 1);
            __syncthreads();
        }
        double acc[KG];
#pragma unroll
        for (int c = 0; c < KG; ++c) {
            double cm = 0.0;
#pragma unroll
            for (int a = 0; a < 4; ++a) cm += phi[a] * S.c[(own_slot * 4 + a) * KG + c];
            m[c] = v[c] + cm;
            acc[c] = 0.0;
        }
        if (act) {
#pragma unroll
            for (int e = 0; e < kCache; ++e)
#pragma unroll
                for (int c = 0; c < KG; ++c) acc[c] += cv[e] * vnb[e][c];
#pragma unroll
            for (int q = 0; q < kPcgRegSlots; ++q)
                if (rsl[q] >= 0) {
#pragma unroll
                    for (int a = 0; a < 4; ++a)
#pragma unroll
                        for (int c = 0; c < KG; ++c) acc[c] += rwt[q][a] * S.c[(rsl[q] * 4 + a) * KG + c];
                }
            for (int q = kPcgRegSlots; q < nq_row; ++q) {   // slots are filled in order
                const int sl = A.rslot[(int64_t)q * n + i];
#pragma unroll
                for (int a = 0; a < 4; ++a) {
                    const double wq = A.rw[((int64_t)q * 4 + a) * n + i];
#pragma unroll
                    for (int c = 0; c < KG; ++c) acc[c] += wq * S.c[(sl * 4 + a) * KG + c];
                }
            }
            for (int e = kCache; e < A.ell_w; ++e) {   // (their coarse part is in rwt)
                const int32_t j = A.pcol[(int64_t)e * n + i];
                const double a = A.pval[(int64_t)e * n + i];
#pragma unroll
                for (int c = 0; c < KG; ++c)
                    if (c < k) acc[c] += a * xload(Vb + (int64_t)j * k + c);
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
            if (c < k) xstore(redb(cp) + (int64_t)B * 3 * k + g * k + c, S.sums[t]);
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
                if (c < k) xstore(A.x + i * k + c, x[c]);
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
                        if (c < k) acc[c] += cv[e] * xload(A.x + (int64_t)cj[e] * k + c);
            for (int e = kCache; e < A.ell_w; ++e) {
                const int32_t j = A.pcol[(int64_t)e * n + i];
                const double a = A.pval[(int64_t)e * n + i];
#pragma unroll
                for (int c = 0; c < KG; ++c)
                    if (c < k) acc[c] += a * xload(A.x + (int64_t)j * k + c);
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
        if (t < KG && t < k) xstore(redb(cp) + (int64_t)B * 3 * k + t, S.sums[t]);
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
    double x0[KG];
#pragma unroll
    for (int c = 0; c < KG; ++c) {
        r[c] = (act && c < k) ? A.b[i * k + c] : 0.0;
        x0[c] = (A.warm && act && c < k) ? A.x[i * k + c] : 0.0;   // read before x is stored
        x[c] = 0.0;
    }
    int total_it = 0;
    constexpr int kMaxRestarts = 6;
    bool have_bb = false;
    if (A.warm) {
        // warm start: |b|^2 (the residual of x = 0) fixes the tolerance, then the solve
        // starts from the residual of the previous solution
        if (!true_residual()) return;
        if (t < KG) {
            my_bb = S.sums[t];
            my_done = (t >= k) || !(my_bb > 0.0);
        }
        have_bb = true;
#pragma unroll
        for (int c = 0; c < KG; ++c) x[c] = x0[c];
        if (!true_residual()) return;
    }
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

hipError_t launch_pcg_setup(const PcgSetup& ps, const double* V, const int32_t* lap_off, const double* lap_val,
                            hipStream_t s)
{
    hipLaunchKernelGGL(k_perm_ell_vals, dim3((unsigned)((ps.n + 255) / 256)), dim3(256), 0, s,
                       ps.n, ps.ell_w, ps.perm, lap_off, lap_val, ps.pval);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // coarse functions, their rows of C and the Galerkin matrix; then both inverses
    hipLaunchKernelGGL(k_agg_basis, dim3(ps.na), dim3(kAggThreads), 0, s, ps.perm, V, ps.astart, ps.bstart, ps.phi,
                       ps.esum);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_row_coarse, dim3((unsigned)((ps.n + 255) / 256)), dim3(256), 0, s, ps.n, ps.ell_w, ps.pcol,
                       ps.pval, ps.eslot, ps.phi, ps.rw);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const int64_t nn = (int64_t)ps.nc * ps.nc;
    hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)((nn + 255) / 256)), dim3(256), 0, s, ps.C0inv, nn);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const size_t asm_smem = sizeof(double) * kAsmGroups * (size_t)ps.na * 16;
    e = hipFuncSetAttribute((const void*)k_coarse_assemble, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)(sizeof(double) * kAsmGroups * (kCoarseMax / 4) * 16));
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_coarse_assemble, dim3(ps.na), dim3(kAggThreads), asm_smem, s, ps.n, ps.na, ps.nc,
                       ps.astart, ps.bstart, ps.blk, ps.abl_off, ps.abl, ps.rslot, ps.phi, ps.rw, ps.C0inv);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const size_t binv_smem = sizeof(double) * kBS * kBS;
    e = hipFuncSetAttribute((const void*)k_inverses, hipFuncAttributeMaxDynamicSharedMemorySize, (int)binv_smem);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_inverses, dim3(ps.nb + 1), dim3(kInvThreads), binv_smem, s, ps.nb, ps.n, ps.ell_w, ps.pcol,
                       ps.pval, ps.bstart, ps.whole, ps.Binv, ps.nc, ps.acomp, ps.esum, ps.C0inv);
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

int pcg_block_size() { return kBS; }
int pcg_max_blocks() { return kMaxNbPcg; }
int pcg_max_coarse() { return kCoarseMax; }
int pcg_max_block_aggregates() { return kMaxAggNbn; }
size_t pcg_table_bytes(int n) { return sizeof(PcgArgs) * (size_t)std::max(n, 1); }

hipError_t launch_pcg_batch(const PcgItem* items, int n, int k, void* tab_dev, void* tab_host,
                            hipStream_t s)
{
    if (n < 1) return hipSuccess;
    const void* fn = pcg_fn(k);
    if (!fn) return hipErrorInvalidValue;
    // LDS staging of the block shares when the largest problem's fit beside PcgShared
    hipError_t e0;
    int nb_max = 0;
    for (int m = 0; m < n; ++m) nb_max = std::max(nb_max, items[m].ps->nb);
    const size_t base = (pcg_smem_bytes(k) + 15) / 16 * 16;
    const size_t stage_bytes = sizeof(double) * (size_t)nb_max * 4 * (size_t)k;
    int lds_max = 0;
    e0 = hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, device_info().device);
    if (e0 != hipSuccess) return e0;
    const bool stage = base + stage_bytes <= (size_t)lds_max;
    const size_t smem = stage ? base + stage_bytes : pcg_smem_bytes(k);
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
        a.n = ps.n; a.nb = ps.nb; a.nc = ps.nc; a.ell_w = ps.ell_w; a.pcol = ps.pcol; a.pval = ps.pval;
        a.bstart = ps.bstart; a.astart = ps.astart; a.agg_of_block = ps.agg_of_block; a.abl_off = ps.abl_off;
        a.abl = ps.abl; a.rslot = ps.rslot; a.phi = ps.phi; a.rw = ps.rw; a.Binv = ps.Binv; a.C0inv = ps.C0inv;
        a.b = it.b; a.x = it.x; a.Vb = it.w.Vb; a.rho = it.w.rho; a.red = it.w.red; a.bar = it.w.bar;
        a.iters = it.w.iters; a.relres = it.w.relres; a.flags = it.w.flags;
        a.rtol = it.rtol; a.maxiter = it.maxiter; a.k = k; a.block0 = 0; a.stage = stage ? 1 : 0;
        a.warm = it.warm ? 1 : 0;
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


// ---------------------------------------------------------------- multi-launch solve
//
// For problems with more blocks than workgroups that can be resident at once, the same
// preconditioned Chronopoulos-Gear iteration runs as one kernel per phase; the kernel
// boundaries are the grid-wide synchronisation.  Per iteration:
//   k_ml_block       the previous iteration's update of the block's rows (p = m + beta p,
//                    s = an + beta s, x += alpha p, r -= alpha s), then v = C_BB^{-1} r_B
//                    (FP32, as in k_pcg) and the block's shares Phi_B^T r
//   k_ml_coarse_rhs  coarse right-hand side g: per aggregate, its blocks' shares in order
//   k_ml_apply       coarse values of the aggregates of the workgroup's rows (rows of
//                    C0^{-1} times g), m = v + Phi c
//   k_ml_spmv        an = C m, partial sums of (r, m), (an, m), (r, r) per workgroup
//   k_ml_scalars     the sums in fixed order, alpha and beta per column, the stop flag
// Every kernel returns at once when the stop flag is set, so a batch of iterations
// enqueued past convergence costs only its launches; the host reads the flag after each
// batch, then verifies with the true residual b - C x and restarts from it when needed.
// The update of an iteration that raised the stop flag is never applied: it has alpha = 0
// in every column, so it would leave x and r as they are.

constexpr int kMlRows = kThreads;     // rows per workgroup of the row-parallel kernels
constexpr int kMlBatch = 16;          // iterations enqueued between two reads of the flag
constexpr int kMlScalarThreads = 1024;

struct MlState {
    int stop, total_it, first, have_bb;
    int upd;                                       // an update is pending (ca, cb)
    int done[kMaxGroupCols], its[kMaxGroupCols];
    double bb[kMaxGroupCols], rr[kMaxGroupCols], gam[kMaxGroupCols], alpha[kMaxGroupCols];
    double ca[kMaxGroupCols], cb[kMaxGroupCols];   // this iteration's alpha, beta (0 when frozen)
};

__global__ void k_ml_init(MlState* st)
{
    if (threadIdx.x == 0) {
        st->stop = 0;
        st->total_it = 0;
        st->first = 1;
        st->have_bb = 0;
        st->upd = 0;
        for (int c = 0; c < kMaxGroupCols; ++c) {
            st->done[c] = 0;
            st->its[c] = 0;
            st->bb[c] = st->rr[c] = st->gam[c] = st->alpha[c] = st->ca[c] = st->cb[c] = 0.0;
        }
    }
}

// r = b - C x (x = 0 when zero_x: then r = b and x is cleared), p = s = 0, and per
// workgroup the partial sums of r^2 (part[wg][0][c]).
template <int KG>
__global__ __launch_bounds__(kMlRows) void k_ml_residual(int64_t n, int k, int w, const int32_t* __restrict__ pcol,
                                                         const double* __restrict__ pval, const double* __restrict__ b,
                                                         double* __restrict__ x, double* __restrict__ r,
                                                         double* __restrict__ p, double* __restrict__ s,
                                                         double* __restrict__ part, int zero_x)
{
    __shared__ double wave_sh[(kMlRows / 64) * KG];
    __shared__ double sums[KG];
    const int64_t i = (int64_t)blockIdx.x * kMlRows + threadIdx.x;
    double rr[KG];
#pragma unroll
    for (int c = 0; c < KG; ++c) rr[c] = 0.0;
    if (i < n) {
        double cx[KG];
#pragma unroll
        for (int c = 0; c < KG; ++c) cx[c] = 0.0;
        if (!zero_x)
            for (int e = 0; e < w; ++e) {
                const int32_t j = pcol[(int64_t)e * n + i];
                const double a = pval[(int64_t)e * n + i];
#pragma unroll
                for (int c = 0; c < KG; ++c)
                    if (c < k) cx[c] += a * x[(int64_t)j * k + c];
            }
#pragma unroll
        for (int c = 0; c < KG; ++c)
            if (c < k) {
                const int64_t id = i * k + c;
                const double rv = b[id] - cx[c];
                if (zero_x) x[id] = 0.0;   // (x is not read when zero_x)
                r[id] = rv;
                p[id] = 0.0;
                s[id] = 0.0;
                rr[c] = rv * rv;
            }
    }
    wg_reduce<KG>(rr, wave_sh, sums);
    if ((int)threadIdx.x < KG) part[(int64_t)blockIdx.x * 3 * KG + threadIdx.x] = sums[threadIdx.x];
}

// The block's rows of r are read and its rows of v written as one contiguous range (the
// row stride is KG), staged through LDS.
template <int KG>
__global__ __launch_bounds__(kThreads) void k_ml_block(const MlState* __restrict__ st,
                                                       const int32_t* __restrict__ bstart,
                                                       const float* __restrict__ Binv, const double* __restrict__ phi,
                                                       const double* __restrict__ m, const double* __restrict__ an,
                                                       double* __restrict__ p, double* __restrict__ s,
                                                       double* __restrict__ x, double* __restrict__ r,
                                                       double* __restrict__ v, double* __restrict__ shares)
{
    __shared__ float r32[kBS * KG];
    __shared__ double y64[kBS * KG];
    __shared__ double half[kBS * KG];
    __shared__ double wave_sh[(kThreads / 64) * 4 * KG];
    __shared__ double sums[4 * KG];
    __shared__ double coef[2 * KG];
    if (st->stop) return;
    const int B = blockIdx.x, t = threadIdx.x;
    const int32_t s0 = bstart[B], cnt = bstart[B + 1] - s0;
    const bool upd = st->upd != 0;
    if (t < KG) {
        coef[t] = st->ca[t];
        coef[KG + t] = st->cb[t];
    }
    __syncthreads();
    const int64_t e0 = (int64_t)s0 * KG;
    for (int e = t; e < kBS * KG; e += kThreads) {
        double yv = 0.0;
        if (e < cnt * KG) {
            const int64_t id = e0 + e;
            yv = r[id];
            if (upd) {
                const int c = e % KG;
                const double al = coef[c], be = coef[KG + c];
                const double pn = m[id] + be * p[id];
                const double sn = an[id] + be * s[id];
                p[id] = pn;
                s[id] = sn;
                x[id] += al * pn;
                yv -= al * sn;
                r[id] = yv;
            }
        }
        y64[e] = yv;
        r32[e] = (float)yv;
    }
    __syncthreads();
    // the block product as in k_pcg: FP32, row tt's sum in two halves of j
    const int tt = t & (kBS - 1), jbeg = (t / kBS) * (kBS / 2);
    const float* Bi = Binv + (int64_t)B * kBS * kBS;
    float v32[KG];
#pragma unroll
    for (int c = 0; c < KG; ++c) v32[c] = 0.0f;
    constexpr int CH = 8;
#pragma unroll 1
    for (int j0 = jbeg; j0 < jbeg + kBS / 2; j0 += CH) {
        float bj[CH], yj[CH * KG];
#pragma unroll
        for (int q = 0; q < CH; ++q) bj[q] = Bi[(j0 + q) * kBS + tt];
#pragma unroll
        for (int q = 0; q < CH * KG; ++q) yj[q] = r32[j0 * KG + q];
#pragma unroll
        for (int q = 0; q < CH; ++q)
#pragma unroll
            for (int c = 0; c < KG; ++c) v32[c] = __builtin_fmaf(bj[q], yj[q * KG + c], v32[c]);
    }
    if (t >= kBS) {
#pragma unroll
        for (int c = 0; c < KG; ++c) half[tt * KG + c] = (double)v32[c];
    }
    __syncthreads();
    if (t < kBS) {
#pragma unroll
        for (int c = 0; c < KG; ++c) half[t * KG + c] += (double)v32[c];   // own half + helper half
    }
    // the block's shares of the coarse right-hand side: sum over its rows of phi[a] y
    double tmp[4 * KG];
    {
        const bool act = t < cnt;
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            const double ph = act ? phi[(int64_t)(s0 + t) * 4 + a] : 0.0;
#pragma unroll
            for (int c = 0; c < KG; ++c) tmp[a * KG + c] = act ? ph * y64[t * KG + c] : 0.0;
        }
    }
    wg_reduce<4 * KG>(tmp, wave_sh, sums);   // (its barriers also order the writes to half)
    if (t < 4 * KG) shares[(int64_t)B * 4 * KG + t] = sums[t];
    double* vb = v + (int64_t)s0 * KG;
    for (int e = t; e < cnt * KG; e += kThreads) vb[e] = half[e];
}

// g[4 ag + a][c] = sum over the blocks of aggregate ag, in order, of their shares.
template <int KG>
__global__ __launch_bounds__(64) void k_ml_coarse_rhs(const MlState* __restrict__ st, const int32_t* __restrict__ astart,
                                                      const double* __restrict__ shares, double* __restrict__ g)
{
    if (st->stop) return;
    const int ag = blockIdx.x, t = threadIdx.x;
    if (t >= 4 * KG) return;
    const int b0 = astart[ag], b1 = astart[ag + 1];
    double acc = 0.0;
    for (int bb = b0; bb < b1; bb += 8) {
        double u[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) u[q] = bb + q < b1 ? shares[(int64_t)(bb + q) * 4 * KG + t] : 0.0;
#pragma unroll
        for (int q = 0; q < 8; ++q) acc += u[q];
    }
    g[(int64_t)ag * 4 * KG + t] = acc;
}

// Coarse values of the aggregates of rows [r0, r0 + kMlRows) (consecutive in block order),
// then m = v + Phi c for those rows.
template <int KG>
__global__ __launch_bounds__(kMlRows) void k_ml_apply(const MlState* __restrict__ st, int64_t n, int nc,
                                                      const int32_t* __restrict__ blk,
                                                      const int32_t* __restrict__ agg_of_block,
                                                      const double* __restrict__ C0inv, const double* __restrict__ g,
                                                      const double* __restrict__ phi, const double* __restrict__ v,
                                                      double* __restrict__ m)
{
    __shared__ double gs[kCoarseMax * KG];
    __shared__ double cw[kCoarseMax * KG];
    __shared__ double psum[kMlRows];
    if (st->stop) return;
    const int t = threadIdx.x;
    const int64_t r0 = (int64_t)blockIdx.x * kMlRows;
    const int64_t r1 = min(n, r0 + kMlRows);
    const int ag_lo = agg_of_block[blk[r0]], ag_hi = agg_of_block[blk[r1 - 1]];
    for (int q = t; q < nc * KG; q += kMlRows) gs[q] = g[q];
    __syncthreads();
    const int jobs = (ag_hi - ag_lo + 1) * 4 * KG;
    for (int j0 = 0; j0 < jobs; j0 += kMlRows) {
        const int nj = min(kMlRows, jobs - j0);
        const int P = max(1, kMlRows / nj);
        const int chunk = (nc + P - 1) / P;
        const int jl = t / P, pt = t - jl * P;
        if (jl < nj) {
            const int job = j0 + jl, row = job / KG, c = job - row * KG;
            const int d = 4 * ag_lo + row;
            const int d0 = pt * chunk, d1 = min(nc, d0 + chunk);
            psum[jl * P + pt] = d1 > d0 ? dot_fixed(C0inv + (int64_t)d * nc + d0, gs + d0 * KG + c, d1 - d0, KG) : 0.0;
        }
        __syncthreads();
        if (t < nj) cw[j0 + t] = sum_fixed(psum + t * P, P, 1);
        __syncthreads();
    }
    // element-wise over the rows' KG columns (contiguous loads and stores)
    for (int64_t e = r0 * KG + t; e < r1 * KG; e += kMlRows) {
        const int64_t i = e / KG;
        const int c = (int)(e - i * KG);
        const int ag = agg_of_block[blk[i]] - ag_lo;
        double cm = 0.0;
#pragma unroll
        for (int a = 0; a < 4; ++a) cm += phi[i * 4 + a] * cw[(ag * 4 + a) * KG + c];
        m[e] = v[e] + cm;
    }
}

// an = C m and the partial sums of (r, m), (an, m), (r, r): one thread per element (row,
// column) of R = kMlSpThreads / KG rows at a time, `rounds` times (chosen at launch so
// that there are about kMlSpTargetWg workgroups: enough to fill the device, few enough
// partial sums for the scalars kernel), the gathers of a row's KG values contiguous across
// lanes; the partial sums go through LDS and are added per column over the rows in order.
constexpr int kMlSpThreads = 1024;
constexpr int kMlSpTargetWg = 384;
constexpr int kMlSpMaxRounds = 4;
template <int KG>
__global__ __launch_bounds__(kMlSpThreads) void k_ml_spmv(const MlState* __restrict__ st, int64_t n, int rounds, int w,
                                                          const int32_t* __restrict__ pcol,
                                                          const double* __restrict__ pval,
                                                          const double* __restrict__ m, const double* __restrict__ r,
                                                          double* __restrict__ an, double* __restrict__ part)
{
    constexpr int R = kMlSpThreads / KG;
    __shared__ double val[3][R * KG];
    if (st->stop) return;
    const int t = threadIdx.x;
    const int64_t r0 = (int64_t)blockIdx.x * R * rounds;
    const int rl = t / KG, c = t - rl * KG;
    double v0 = 0.0, v1 = 0.0, v2 = 0.0;   // this thread's column, its rows added in order
    for (int rd = 0; rd < rounds; ++rd) {
        const int64_t i = r0 + (int64_t)rd * R + rl;
        if (rl < R && i < n) {
            double acc = 0.0;
            for (int e = 0; e < w; ++e) {
                const int32_t j = pcol[(int64_t)e * n + i];
                acc += pval[(int64_t)e * n + i] * m[(int64_t)j * KG + c];
            }
            const int64_t id = i * KG + c;
            const double mi = m[id], ri = r[id];
            an[id] = acc;
            v0 += ri * mi;
            v1 += acc * mi;
            v2 += ri * ri;
        }
    }
    if (rl < R) {
        val[0][t] = v0;
        val[1][t] = v1;
        val[2][t] = v2;
    }
    __syncthreads();
    // each of the 3 KG sums over the R rows in P parts of consecutive rows, then the parts
    // in order
    constexpr int M = 3 * KG, P = kMlSpThreads / M, CH = (R + P - 1) / P;
    __shared__ double ps[kMlSpThreads];
    {
        const int q = t / P, pt = t - q * P;
        if (q < M) {
            const int g = q / KG, cc = q - g * KG;
            const int ro0 = pt * CH, ro1 = min(R, ro0 + CH);
            double acc = 0.0;
            for (int ro = ro0; ro < ro1; ++ro) acc += val[g][ro * KG + cc];
            ps[q * P + pt] = acc;
        }
    }
    __syncthreads();
    if (t < M) {
        double a = 0.0;
        for (int z = 0; z < P; ++z) a += ps[t * P + z];
        part[(int64_t)blockIdx.x * 3 * KG + t] = a;
    }
}

// Sums over the nwg workgroups of the first M values of part ([nwg][3KG]) in a fixed
// order (each value cut into P parts of consecutive workgroups, the parts added in order)
// into tot[0 .. M), by kMlScalarThreads threads.
template <int M, int KG>
__device__ __forceinline__ void ml_grid_sum(const double* __restrict__ part, int nwg, double* ps, double* tot)
{
    constexpr int P = kMlScalarThreads / M;
    const int t = threadIdx.x;
    const int chunk = (nwg + P - 1) / P;
    const int q = t / P, pt = t - q * P;
    if (q < M) {
        const int w0 = pt * chunk, w1 = min(nwg, w0 + chunk);
        double acc = 0.0;
        for (int ww = w0; ww < w1; ww += 8) {
            double u[8];
#pragma unroll
            for (int z = 0; z < 8; ++z) u[z] = ww + z < w1 ? part[(int64_t)(ww + z) * 3 * KG + q] : 0.0;
#pragma unroll
            for (int z = 0; z < 8; ++z) acc += u[z];
        }
        ps[q * P + pt] = acc;
    }
    __syncthreads();
    if (t < M) {
        double a = 0.0;
        for (int z = 0; z < P; ++z) a += ps[t * P + z];
        tot[t] = a;
    }
    __syncthreads();
}

// The column scalars of one iteration (the rules of k_pcg): gamma = (r, m), delta =
// (an, m), |r|^2; the first iteration of a solve takes |b|^2 from it; columns whose |r|^2
// is at or below rtol^2 |b|^2 are frozen (alpha = beta = 0); the stop flag is raised when
// no column is open or the iteration budget is spent.
template <int KG>
__global__ __launch_bounds__(kMlScalarThreads) void k_ml_scalars(MlState* __restrict__ st, const double* __restrict__ part,
                                                                  int nwg, int k, double rtol2, int maxiter)
{
    __shared__ double ps[kMlScalarThreads];
    __shared__ double tot[3 * KG];
    __shared__ int live_sh[KG];
    if (st->stop) return;
    ml_grid_sum<3 * KG, KG>(part, nwg, ps, tot);
    const int t = threadIdx.x;
    const bool can = st->total_it < maxiter;
    if (t < KG) {
        const int c = t;
        const double gm = tot[c], de = tot[KG + c], rrv = tot[2 * KG + c];
        if (!st->have_bb) {
            st->bb[c] = rrv;
            st->done[c] = (c >= k || !(rrv > 0.0)) ? 1 : 0;
        }
        st->rr[c] = rrv;
        const bool live = !st->done[c] && rrv > rtol2 * st->bb[c];
        double al = 0.0, be = 0.0;
        if (live) {
            if (can) {
                if (st->first) {
                    al = gm / de;
                } else {
                    be = gm / st->gam[c];
                    al = gm / (de - be * gm / st->alpha[c]);
                }
                st->its[c] = st->total_it + 1;
            }
            st->gam[c] = gm;
            st->alpha[c] = al;
        }
        st->ca[c] = al;
        st->cb[c] = be;
        live_sh[c] = live ? 1 : 0;
    }
    __syncthreads();
    if (t == 0) {
        bool any = false;
        for (int c = 0; c < KG; ++c) any = any || live_sh[c] != 0;
        st->have_bb = 1;
        if (!any || !can) {
            st->stop = 1;
        } else {
            st->total_it += 1;
            st->first = 0;
            st->upd = 1;
        }
    }
}

// After a true residual (k_ml_residual): columns at or below rtol^2 |b|^2 are done; the
// solve ends when all are done or the budget is spent, else it restarts from r (the stop
// flag is lowered and the next iteration is a first one).
template <int KG>
__global__ __launch_bounds__(kMlScalarThreads) void k_ml_verify(MlState* __restrict__ st, const double* __restrict__ part,
                                                                 int nwg, double rtol2, int maxiter)
{
    __shared__ double ps[kMlScalarThreads];
    __shared__ double tot[KG];
    ml_grid_sum<KG, KG>(part, nwg, ps, tot);
    const int t = threadIdx.x;
    if (t < KG && !st->done[t]) {
        st->rr[t] = tot[t];
        if (tot[t] <= rtol2 * st->bb[t]) st->done[t] = 1;
    }
    __syncthreads();
    if (t == 0) {
        bool all = true;
        for (int c = 0; c < KG; ++c) all = all && st->done[c] != 0;
        st->upd = 0;
        if (all || st->total_it >= maxiter) {
            st->stop = 1;
        } else {
            st->stop = 0;
            st->first = 1;
        }
    }
}

__global__ void k_ml_finish(const MlState* __restrict__ st, int k, int* __restrict__ iters, double* __restrict__ relres)
{
    const int c = threadIdx.x;
    if (c < k) {
        iters[c] = st->its[c];
        relres[c] = st->bb[c] > 0.0 ? sqrt(st->rr[c] / st->bb[c]) : 0.0;
    }
}

namespace {

template <int KG>
hipError_t launch_pcg_ml_k(const PcgSetup& ps, const double* b, double* x, int k, double rtol, int maxiter,
                           const PcgMlWork& w, int* iters, double* relres, hipStream_t s)
{
    const int64_t n = ps.n;
    const int nwg = (int)((n + kMlRows - 1) / kMlRows);
    constexpr int kSpR = kMlSpThreads / KG;
    const int sp_rounds = (int)std::max<int64_t>(1, std::min<int64_t>(kMlSpMaxRounds, (n + kSpR - 1) / kSpR / kMlSpTargetWg));
    const int64_t sp_rows = (int64_t)kSpR * sp_rounds;
    const int nws = (int)((n + sp_rows - 1) / sp_rows);
    if (k != KG) return hipErrorInvalidValue;
    MlState* st = static_cast<MlState*>(w.state);
    MlState* hs = static_cast<MlState*>(w.state_host);
    const double rtol2 = rtol * rtol;
    hipError_t e;
#define TP_ML_CHECK() do { if ((e = hipGetLastError()) != hipSuccess) return e; } while (0)
    hipLaunchKernelGGL(k_ml_init, dim3(1), dim3(64), 0, s, st);
    TP_ML_CHECK();
    hipLaunchKernelGGL((k_ml_residual<KG>), dim3(nwg), dim3(kMlRows), 0, s, n, k, ps.ell_w, ps.pcol, ps.pval, b, x,
                       w.r, w.p, w.s, w.part, 1);
    TP_ML_CHECK();
    constexpr int kMaxRestarts = 6;
    for (int cycle = 0;; ++cycle) {
        for (;;) {
            for (int q = 0; q < kMlBatch; ++q) {
                hipLaunchKernelGGL((k_ml_block<KG>), dim3(ps.nb), dim3(kThreads), 0, s, st, ps.bstart, ps.Binv,
                                   ps.phi, w.m, w.an, w.p, w.s, x, w.r, w.v, w.shares);
                hipLaunchKernelGGL((k_ml_coarse_rhs<KG>), dim3(ps.na), dim3(64), 0, s, st, ps.astart, w.shares, w.g);
                hipLaunchKernelGGL((k_ml_apply<KG>), dim3(nwg), dim3(kMlRows), 0, s, st, n, ps.nc, ps.blk,
                                   ps.agg_of_block, ps.C0inv, w.g, ps.phi, w.v, w.m);
                hipLaunchKernelGGL((k_ml_spmv<KG>), dim3(nws), dim3(kMlSpThreads), 0, s, st, n, sp_rounds, ps.ell_w, ps.pcol,
                                   ps.pval, w.m, w.r, w.an, w.part);
                hipLaunchKernelGGL((k_ml_scalars<KG>), dim3(1), dim3(kMlScalarThreads), 0, s, st, w.part, nws, k,
                                   rtol2, maxiter);
            }
            TP_ML_CHECK();
            if ((e = hipMemcpyAsync(hs, st, sizeof(MlState), hipMemcpyDeviceToHost, s)) != hipSuccess) return e;
            if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
            if (hs->stop) break;
        }
        // true residual, then verification (and a restart from it when needed)
        hipLaunchKernelGGL((k_ml_residual<KG>), dim3(nwg), dim3(kMlRows), 0, s, n, k, ps.ell_w, ps.pcol, ps.pval, b,
                           x, w.r, w.p, w.s, w.part, 0);
        hipLaunchKernelGGL((k_ml_verify<KG>), dim3(1), dim3(kMlScalarThreads), 0, s, st, w.part, nwg, rtol2, maxiter);
        TP_ML_CHECK();
        if ((e = hipMemcpyAsync(hs, st, sizeof(MlState), hipMemcpyDeviceToHost, s)) != hipSuccess) return e;
        if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
        if (hs->stop || cycle >= kMaxRestarts) break;
    }
    hipLaunchKernelGGL(k_ml_finish, dim3(1), dim3(64), 0, s, st, k, iters, relres);
    TP_ML_CHECK();
#undef TP_ML_CHECK
    return hipSuccess;
}

}  // namespace

int pcg_max_blocks_multi() { return kMaxNbMulti; }
size_t pcg_ml_state_bytes() { return sizeof(MlState); }
// per-workgroup partial sums: the residual kernel's kMlRows rows per workgroup or the
// sparse product's one round of kMlSpThreads / KG rows, whichever gives more workgroups
size_t pcg_ml_part_doubles(int64_t n)
{
    const int64_t rows = std::min<int64_t>(kMlRows, kMlSpThreads / kMaxGroupCols);
    return (size_t)((n + rows - 1) / rows) * 3 * kMaxGroupCols;
}

hipError_t launch_pcg_ml(const PcgSetup& ps, const double* b, double* x, int k, double rtol, int maxiter,
                         const PcgMlWork& w, int* iters, double* relres, hipStream_t s)
{
    switch (k) {
    case 1: return launch_pcg_ml_k<1>(ps, b, x, k, rtol, maxiter, w, iters, relres, s);
    case 2: return launch_pcg_ml_k<2>(ps, b, x, k, rtol, maxiter, w, iters, relres, s);
    case 3: return launch_pcg_ml_k<3>(ps, b, x, k, rtol, maxiter, w, iters, relres, s);
    case 4: return launch_pcg_ml_k<4>(ps, b, x, k, rtol, maxiter, w, iters, relres, s);
    case 5: return launch_pcg_ml_k<5>(ps, b, x, k, rtol, maxiter, w, iters, relres, s);
    case 6: return launch_pcg_ml_k<6>(ps, b, x, k, rtol, maxiter, w, iters, relres, s);
    case 7: return launch_pcg_ml_k<7>(ps, b, x, k, rtol, maxiter, w, iters, relres, s);
    case 8: return launch_pcg_ml_k<8>(ps, b, x, k, rtol, maxiter, w, iters, relres, s);
    case 9: return launch_pcg_ml_k<9>(ps, b, x, k, rtol, maxiter, w, iters, relres, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace tp
