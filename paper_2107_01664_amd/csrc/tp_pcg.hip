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
// The solver is the Chronopoulos-Gear form of preconditioned CG: u = M^{-1} r, w = C u,
// gamma = (r, u), delta = (w, u).  One workgroup of kBS threads owns one block (one row per
// thread) and keeps its C_BB^{-1} in LDS for the whole solve.  Each iteration has two
// grid exchanges (two-level counter barriers, bounded spins):
//   A. after x, r, p, s updates: the block solve v = C_BB^{-1} r_B, the block sums of r
//      (coarse right-hand side) and sum r^2 are published;
//   B. after w = C u with u = v + c(block), where the coarse values c of the own and the
//      neighbouring blocks are formed from the published block sums: (r,u), (w,u).
// All partial sums are added in block order by every workgroup, so every workgroup takes
// the same decisions and the result does not depend on scheduling.
#include "tp_internal.h"

#include <algorithm>
#include <type_traits>
#include <utility>
#include <vector>

namespace tp {

constexpr int kBS = 128;            // vertices per block = threads per solver workgroup
constexpr int kMaxNbn = 32;         // neighbouring blocks of a block (itself included)
constexpr int kMaxNbPcg = 256;      // blocks (one co-resident workgroup per block)

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
__global__ __launch_bounds__(256) void k_block_inverse(int64_t n, int w, const int32_t* __restrict__ pcol,
                                                       const double* __restrict__ pval,
                                                       const int32_t* __restrict__ bstart,
                                                       const int32_t* __restrict__ whole,
                                                       float* __restrict__ Binv)
{
    extern __shared__ __align__(16) double A[];   // kBS x kBS, row-major
    __shared__ double fcol[kBS];
    const int B = blockIdx.x;
    const int32_t s0 = bstart[B], cnt = bstart[B + 1] - s0;
    for (int t = threadIdx.x; t < kBS * kBS; t += blockDim.x) A[t] = 0.0;
    __syncthreads();
    for (int t = threadIdx.x; t < kBS; t += blockDim.x) {
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
        for (int t = threadIdx.x; t < cnt * cnt; t += blockDim.x) A[(t / cnt) * kBS + (t % cnt)] += add;
        __syncthreads();
    }
    for (int k = 0; k < kBS; ++k) {
        const double p = 1.0 / A[k * kBS + k];
        __syncthreads();
        for (int j = threadIdx.x; j < kBS; j += blockDim.x) {
            fcol[j] = A[j * kBS + k];           // column k before the update
        }
        __syncthreads();
        for (int j = threadIdx.x; j < kBS; j += blockDim.x)
            A[k * kBS + j] = (j == k ? 1.0 : A[k * kBS + j]) * p;
        __syncthreads();
        for (int t = threadIdx.x; t < kBS * kBS; t += blockDim.x) {
            const int i = t / kBS, j = t - i * kBS;
            if (i != k) {
                const double base = (j == k) ? 0.0 : A[i * kBS + j];
                A[i * kBS + j] = base - fcol[i] * A[k * kBS + j];
            }
        }
        __syncthreads();
    }
    // symmetrize (the elimination leaves rounding-level asymmetry) and round to FP32
    float* dst = Binv + (int64_t)B * kBS * kBS;
    for (int t = threadIdx.x; t < kBS * kBS; t += blockDim.x) {
        const int i = t / kBS, j = t - i * kBS;
        dst[t] = (float)(0.5 * (A[i * kBS + j] + A[j * kBS + i]));
    }
}

// Coarse matrix rows: C0[B][B'] = sum over rows of B of the entries in columns of B'.
// One workgroup per block; thread 0 adds in row order (deterministic).
__global__ __launch_bounds__(64) void k_coarse_rows(int64_t n, int w, int nb, const int32_t* __restrict__ pcol,
                                                    const double* __restrict__ pval,
                                                    const int32_t* __restrict__ bstart,
                                                    const int32_t* __restrict__ blk,
                                                    double* __restrict__ C0)
{
    extern __shared__ __align__(16) double acc[];   // nb
    const int B = blockIdx.x;
    for (int t = threadIdx.x; t < nb; t += blockDim.x) acc[t] = 0.0;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int64_t i = bstart[B]; i < bstart[B + 1]; ++i)
            for (int e = 0; e < w; ++e) acc[blk[pcol[(int64_t)e * n + i]]] += pval[(int64_t)e * n + i];
    }
    __syncthreads();
    for (int t = threadIdx.x; t < nb; t += blockDim.x) C0[(int64_t)B * nb + t] = acc[t];
}

// In-place Gauss-Jordan inverse of the nb x nb coarse matrix (one workgroup, global
// memory), after adding the per-component rank-one terms.
__global__ __launch_bounds__(1024) void k_coarse_inverse(int nb, const int32_t* __restrict__ bcomp,
                                                         const int32_t* __restrict__ ncomp_blocks,
                                                         double* __restrict__ A)
{
    __shared__ double fcol[kMaxNbPcg];
    __shared__ double dmean;
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int i = 0; i < nb; ++i) s += A[(int64_t)i * nb + i];
        dmean = s / nb;
    }
    __syncthreads();
    for (int t = threadIdx.x; t < nb * nb; t += blockDim.x) {
        const int i = t / nb, j = t - i * nb;
        if (bcomp[i] == bcomp[j]) A[t] += dmean / ncomp_blocks[bcomp[i]];
    }
    __syncthreads();
    for (int k = 0; k < nb; ++k) {
        const double p = 1.0 / A[(int64_t)k * nb + k];
        __syncthreads();
        for (int j = threadIdx.x; j < nb; j += blockDim.x) fcol[j] = A[(int64_t)j * nb + k];
        __syncthreads();
        for (int j = threadIdx.x; j < nb; j += blockDim.x)
            A[(int64_t)k * nb + j] = (j == k ? 1.0 : A[(int64_t)k * nb + j]) * p;
        __threadfence_block();
        __syncthreads();
        for (int t = threadIdx.x; t < nb * nb; t += blockDim.x) {
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
    double* Vb;               // [n][k] local solves
    double* rho;              // [nb][k] block sums of r
    double* red;              // [2][nb][2k] block partial sums, buffer = barrier count % 2
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
    double wave[2 * 4 * KG];
    double sums[4 * KG];
    double part[kBS];
    int32_t nbl[kMaxNbn];
};

// Fixed-order workgroup reduction of M values per thread (kBS = 128 threads, two waves):
// butterfly within each wave, then wave 0 + wave 1.  Result in out[0 .. M).
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
    if ((int)threadIdx.x < M) out[threadIdx.x] = wave_sh[threadIdx.x] + wave_sh[M + threadIdx.x];
    __syncthreads();
}

// One launch solves the systems of ntab independent problems: problem m owns workgroups
// [tab[m].block0, tab[m + 1].block0) and synchronises only among them (its own barrier
// words), so its iterates are those of a launch of its own.
template <int KG>
__global__ __launch_bounds__(kBS) void k_pcg(const PcgArgs* __restrict__ tab, int ntab)
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
    const int t = threadIdx.x;
    const bool act = t < cnt;
    const int64_t i = s0 + t;

    {
        const float4* src = reinterpret_cast<const float4*>(A.Binv + (int64_t)B * kBS * kBS);
        float4* dst = reinterpret_cast<float4*>(S.Binv);
        for (int q = t; q < kBS * kBS / 4; q += kBS) dst[q] = src[q];
    }
    const int nbo = A.badj_off[B], nbn = A.badj_off[B + 1] - nbo;
    for (int q = t; q < nbn; q += kBS) S.nbl[q] = A.badj[nbo + q];
    __syncthreads();
    // rows of C0inv for the neighbouring blocks stay in LDS when they fit
    const bool crow_lds = (int64_t)nbn * nb <= kCrowMax;
    if (crow_lds)
        for (int q = t; q < nbn * nb; q += kBS) S.crow[q] = A.C0inv[(int64_t)S.nbl[q / nb] * nb + (q % nb)];
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

    // Sums over all blocks (block order is fixed by the reduction tree): thread t adds
    // blocks t and t + kBS of the published [nb][M/KG][k] array.
    // Partial sums for the m-th barrier go to buffer m % 2: a buffer is rewritten only after
    // the next barrier, by which time every reader of it has arrived there.
    int bcount = 0;
    auto redbuf = [&]() { return A.red + (int64_t)(bcount & 1) * nb * 2 * k; };
    auto grid_sum = [&](auto mtag) {
        // M sums over nb blocks: each value is cut into P parts of consecutive blocks, one
        // per thread (all loads in flight at once), then the parts are added in order.
        constexpr int M = decltype(mtag)::value;
        const double* red = redbuf();
        constexpr int P = kBS / M;
        const int chunk = (nb + P - 1) / P;
        const int q = t / P, part = t - q * P;
        if (q < M) {
            const int g = q / KG, c = q - g * KG;
            double acc = 0.0;
            if (c < k) {
                const int b0 = part * chunk, b1 = min(nb, b0 + chunk);
                for (int bb = b0; bb < b1; ++bb) acc += red[(int64_t)bb * 2 * k + g * k + c];
            }
            S.part[q * P + part] = acc;
        }
        __syncthreads();
        if (t < M) {
            double acc = 0.0;
            for (int pp = 0; pp < P; ++pp) acc += S.part[t * P + pp];
            S.sums[t] = acc;
        }
        __syncthreads();
        ++bcount;
    };

    double r[KG], x[KG], p[KG], s[KG], u[KG], w[KG], v[KG];

    // A: v = C_BB^{-1} r_B; publish v, block sums of r and r^2
    auto phase_a = [&]() {
#pragma unroll
        for (int c = 0; c < KG; ++c) S.r[t * KG + c] = (act && c < k) ? r[c] : 0.0;
        __syncthreads();
#pragma unroll
        for (int c = 0; c < KG; ++c) v[c] = 0.0;
        // padding rows of the block hold r = 0 and an identity block in C_BB^{-1}, so the
        // product runs over all kBS rows with a fixed trip count
#pragma unroll 8
        for (int j = 0; j < kBS; ++j) {
            const double bij = (double)S.Binv[j * kBS + t];
#pragma unroll
            for (int c = 0; c < KG; ++c) v[c] += bij * S.r[j * KG + c];
        }
        double tmp[2 * KG];
#pragma unroll
        for (int c = 0; c < KG; ++c) {
            tmp[c] = act ? r[c] : 0.0;
            tmp[KG + c] = act ? r[c] * r[c] : 0.0;
        }
        wg_reduce<2 * KG>(tmp, S.wave, S.sums);
        if (act)
#pragma unroll
            for (int c = 0; c < KG; ++c)
                if (c < k) A.Vb[i * k + c] = v[c];
        if (t < KG && t < k) {
            A.rho[(int64_t)B * k + t] = S.sums[t];
            redbuf()[(int64_t)B * 2 * k + t] = S.sums[t];
            redbuf()[(int64_t)B * 2 * k + k + t] = S.sums[KG + t];
        }
    };

    // B: coarse values of the own and neighbouring blocks, u = v + c, w = C u; publish
    // block sums of (r,u) and (w,u)
    auto phase_b = [&]() {
        for (int q = t; q < nb * KG; q += kBS) {
            const int bb = q / KG, c = q - bb * KG;
            S.rho[q] = c < k ? A.rho[(int64_t)bb * k + c] : 0.0;
        }
        __syncthreads();
        // coarse values c(sl) = sum_bb C0inv[nbl[sl]][bb] rho[bb] for the nbn x KG jobs: each
        // job's dot product is cut into P parts of consecutive blocks (one per thread)
        const int jobs = nbn * KG;
        for (int j0 = 0; j0 < jobs; j0 += kBS) {
            const int nj = min(kBS, jobs - j0);
            const int P = max(1, kBS / nj);
            const int chunk = (nb + P - 1) / P;
            const int jl = t / P, part = t - jl * P;
            if (jl < nj) {
                const int job = j0 + jl, sl = job / KG, c = job - sl * KG;
                const double* row = crow_lds ? S.crow + sl * nb : A.C0inv + (int64_t)S.nbl[sl] * nb;
                const int b0 = part * chunk, b1 = min(nb, b0 + chunk);
                double acc = 0.0;
                for (int bb = b0; bb < b1; ++bb) acc += row[bb] * S.rho[bb * KG + c];
                S.part[jl * P + part] = acc;
            }
            __syncthreads();
            if (t < nj) {
                double acc = 0.0;
                for (int pp = 0; pp < P; ++pp) acc += S.part[t * P + pp];
                S.c[j0 + t] = acc;
            }
            __syncthreads();
        }
        double acc[KG];
#pragma unroll
        for (int c = 0; c < KG; ++c) {
            u[c] = v[c] + S.c[own_slot * KG + c];
            acc[c] = 0.0;
        }
        if (act) {
#pragma unroll
            for (int e = 0; e < kCache; ++e) {
                if (e < A.ell_w) {
                    const double* vj = A.Vb + (int64_t)cj[e] * k;
#pragma unroll
                    for (int c = 0; c < KG; ++c)
                        if (c < k) acc[c] += cv[e] * (vj[c] + S.c[cs[e] * KG + c]);
                }
            }
            for (int e = kCache; e < A.ell_w; ++e) {
                const int32_t j = A.pcol[(int64_t)e * n + i];
                const double a = A.pval[(int64_t)e * n + i];
                const int sl = A.pslot[(int64_t)e * n + i];
#pragma unroll
                for (int c = 0; c < KG; ++c)
                    if (c < k) acc[c] += a * (A.Vb[(int64_t)j * k + c] + S.c[sl * KG + c]);
            }
        }
        double tmp[2 * KG];
#pragma unroll
        for (int c = 0; c < KG; ++c) {
            w[c] = acc[c];
            tmp[c] = act ? r[c] * u[c] : 0.0;
            tmp[KG + c] = act ? w[c] * u[c] : 0.0;
        }
        wg_reduce<2 * KG>(tmp, S.wave, S.sums);
        if (t < 2 * KG) {
            const int c = t % KG;
            if (c < k) redbuf()[(int64_t)B * 2 * k + (t / KG) * k + c] = S.sums[t];
        }
    };

    // true residual r = b - C x (x published to A.x before the call); block sums of r^2
    auto true_residual = [&]() {
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
        if (t < KG && t < k) redbuf()[(int64_t)B * 2 * k + t] = S.sums[t];
    };

    using C1 = std::integral_constant<int, KG>;
    using C2 = std::integral_constant<int, 2 * KG>;

    double bb[KG], rr[KG], gam[KG], alpha[KG], beta[KG];
    bool done[KG];
    int its[KG];
#pragma unroll
    for (int c = 0; c < KG; ++c) {
        r[c] = (act && c < k) ? A.b[i * k + c] : 0.0;
        x[c] = 0.0;
        its[c] = 0;
        bb[c] = 0.0;
        done[c] = false;
    }
    int total_it = 0;
    constexpr int kMaxRestarts = 6;
    for (int cycle = 0; cycle <= kMaxRestarts; ++cycle) {
        // ---- start of a cycle from the current (true) residual r
#pragma unroll
        for (int c = 0; c < KG; ++c) p[c] = s[c] = 0.0;
        phase_a();
        if (!group_barrier(A.bar, B, nb, A.flags)) return;
        grid_sum(C2{});
        bool all = true;
#pragma unroll
        for (int c = 0; c < KG; ++c) {
            rr[c] = S.sums[KG + c];
            if (cycle == 0) {
                bb[c] = rr[c];
                done[c] = (c >= k) || !(bb[c] > 0.0);
            }
            if (!done[c] && sqrt(rr[c] / bb[c]) <= A.rtol) done[c] = true;
            all = all && done[c];
        }
        __syncthreads();
        if (all || total_it >= A.maxiter) break;
        phase_b();
        if (!group_barrier(A.bar, B, nb, A.flags)) return;
        grid_sum(C2{});
#pragma unroll
        for (int c = 0; c < KG; ++c) {
            gam[c] = S.sums[c];
            alpha[c] = done[c] ? 0.0 : gam[c] / S.sums[KG + c];
            beta[c] = 0.0;
        }
        __syncthreads();
        // ---- iterations
        bool conv = false;
        while (total_it < A.maxiter) {
            ++total_it;
#pragma unroll
            for (int c = 0; c < KG; ++c) {
                p[c] = u[c] + beta[c] * p[c];
                s[c] = w[c] + beta[c] * s[c];
                x[c] += alpha[c] * p[c];
                r[c] -= alpha[c] * s[c];
            }
            phase_a();
            if (!group_barrier(A.bar, B, nb, A.flags)) return;
            grid_sum(C2{});
            conv = true;
#pragma unroll
            for (int c = 0; c < KG; ++c) {
                if (!done[c]) {
                    rr[c] = S.sums[KG + c];
                    its[c] = total_it;
                    if (sqrt(rr[c] / bb[c]) <= A.rtol) {
                        alpha[c] = beta[c] = 0.0;   // column frozen until verified
                    } else {
                        conv = false;
                    }
                }
            }
            __syncthreads();
            if (conv) break;
            phase_b();
            if (!group_barrier(A.bar, B, nb, A.flags)) return;
            grid_sum(C2{});
#pragma unroll
            for (int c = 0; c < KG; ++c) {
                if (!done[c] && sqrt(rr[c] / bb[c]) > A.rtol) {
                    const double gn = S.sums[c], dn = S.sums[KG + c];
                    const double bn = gn / gam[c];
                    alpha[c] = gn / (dn - bn * gn / alpha[c]);
                    beta[c] = bn;
                    gam[c] = gn;
                }
            }
            __syncthreads();
        }
        // ---- verify: publish x, recompute the true residual, restart if needed
        if (act)
#pragma unroll
            for (int c = 0; c < KG; ++c)
                if (c < k) A.x[i * k + c] = x[c];
        if (!group_barrier(A.bar, B, nb, A.flags)) return;
        ++bcount;
        true_residual();
        if (!group_barrier(A.bar, B, nb, A.flags)) return;
        grid_sum(C1{});
        all = true;
#pragma unroll
        for (int c = 0; c < KG; ++c) {
            if (!done[c]) {
                rr[c] = S.sums[c];
                if (sqrt(rr[c] / bb[c]) <= A.rtol) done[c] = true;
            }
            all = all && done[c];
        }
        __syncthreads();
        if (all || total_it >= A.maxiter) break;
    }
    if (act)
#pragma unroll
        for (int c = 0; c < KG; ++c)
            if (c < k) A.x[i * k + c] = x[c];
    if (B == 0 && t < k) {
        A.iters[t] = its[t];
        A.relres[t] = bb[t] > 0.0 ? sqrt(rr[t] / bb[t]) : 0.0;
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
    hipLaunchKernelGGL(k_coarse_rows, dim3(ps.nb), dim3(64), sizeof(double) * ps.nb, s, ps.n, ps.ell_w,
                       ps.nb, ps.pcol, ps.pval, ps.bstart, ps.blk, ps.C0inv);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_coarse_inverse, dim3(1), dim3(1024), 0, s, ps.nb, ps.bcomp, ps.ncomp_blocks, ps.C0inv);
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
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kBS, smem);
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
        e = hipLaunchCooperativeKernel(fn, dim3(blocks), dim3(kBS), params, smem, s);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace tp
