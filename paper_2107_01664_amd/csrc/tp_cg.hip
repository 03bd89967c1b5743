// Persistent FP64 conjugate gradients for the Poisson solves of the preconditioner
// (Sec. 5.2: A~^{-1} = C^{-1} L^sigma C^{-1}, with C the cotan stiffness matrix).
//
// The recurrence is Chronopoulos-Gear CG: both inner products of an iteration,
// gamma = (r, r) and delta = (w, r) with w = C r, come from one reduction, so an iteration
// needs a single grid-wide exchange:
//   p_i = r_i + beta_i p_{i-1},  s_i = w_i + beta_i s_{i-1}   (s_i = C p_i)
//   x_{i+1} = x_i + alpha_i p_i, r_{i+1} = r_i - alpha_i s_i, w_{i+1} = C r_{i+1}
//   beta_{i+1} = gamma_{i+1} / gamma_i,
//   alpha_{i+1} = gamma_{i+1} / (delta_{i+1} - beta_{i+1} gamma_{i+1} / alpha_i).
// The sparse product needs r_{i+1} at neighbouring rows owned by other workgroups; it is
// formed on the fly as r_i - alpha_i (w_i + beta_i s_{i-1}) from the previous iteration's
// values, which sit in one of two buffers (ping-pong by iteration parity), so no
// workgroup overwrites what another may still read and no second barrier is needed.
//
// Layout: the matrix in column-major ELL (width = longest row, padded with the row's own
// index and value 0); per row the state (r, w, s) of all k columns is contiguous,
// Z[buf][row][3][k].  One thread per row handles all columns of its group.  Columns are
// split into groups (blockIdx % ngroups); workgroups of a group meet at a two-level
// counter barrier in global memory (agent-scope atomics) with bounded spins: a wait that
// lasts too long raises an abort flag and every workgroup leaves the loop.  All
// workgroups add the per-workgroup partial sums in the same order, so they take the same
// decisions and the result does not depend on scheduling.
#include "tp_solver.h"

#include <algorithm>

namespace tp {

constexpr int kCgBlock = 256;
constexpr int kMaxW = 256;           // workgroups per column group
static_assert(kMaxW <= kMaxBarrierW, "one barrier flag per workgroup");
constexpr int kMaxGroups = 8;

struct CgArgs {
    int64_t n;
    int ell_w;
    const int32_t* ecol;   // [ell_w][n]
    const double* eval;    // [ell_w][n]
    const double* b;       // [n][k]
    double* x;             // [n][k]
    double* Z;             // [2][n][3][k]
    double* p;             // [n][k]
    double* red;           // [ngroups][2][W][2][KG]
    unsigned* bar;         // [ngroups][kBarWordsPerGroup]
    int* iters;
    double* relres;
    int* flags;
    double rtol;
    int maxiter;
    int k;
    int ngroups;
    int W;
    int rows_per_thread;
};

// Workgroup sums of two KG-vectors (fixed butterfly, then waves in order) into sh_out.
template <int KG>
__device__ __forceinline__ void block_sums2(const double (&a)[KG], const double (&b)[KG],
                                            double* sh_wave, double* sh_out)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int c = 0; c < 2 * KG; ++c) {
        double s = c < KG ? a[c] : b[c - KG];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
        if (lane == 0) sh_wave[wave * 2 * KG + c] = s;
    }
    __syncthreads();
    if (threadIdx.x < 2 * KG) {
        double s = 0.0;
        for (int w = 0; w < kCgBlock / 64; ++w) s += sh_wave[w * 2 * KG + threadIdx.x];
        sh_out[threadIdx.x] = s;
    }
    __syncthreads();
}

template <int KG>
__global__ __launch_bounds__(kCgBlock) void k_cg(CgArgs A)
{
    __shared__ double sh_wave[(kCgBlock / 64) * 2 * KG];
    __shared__ double sh_sum[2 * KG];
    __shared__ double sh_grp[2 * KG];

    const int g = blockIdx.x % A.ngroups;
    const int w = blockIdx.x / A.ngroups;
    const int c0 = g * KG;
    const int nc = min(KG, A.k - c0);
    const int k = A.k;
    const int64_t n = A.n;
    const int64_t rows_per_wg = (int64_t)kCgBlock * A.rows_per_thread;
    const int64_t rb = (int64_t)w * rows_per_wg;
    const int64_t re = min(n, rb + rows_per_wg);
    unsigned* gbar = A.bar + (int64_t)g * kBarWordsPerGroup;
    double* redg = A.red + (int64_t)g * 2 * A.W * 2 * KG;
    const int64_t zrow = 3 * (int64_t)k;             // doubles per row of Z
    double* Z0 = A.Z;
    double* Z1 = A.Z + n * zrow;

    // Group-wide sums of the per-workgroup partials: every thread loads its share of the
    // W x 2KG partials at once, then thread c adds column c over the workgroups in order.
    __shared__ double sh_red[kMaxW * 2 * KG];
    auto group_sum = [&](const double* red) {
        const int tot = A.W * 2 * KG;
        for (int t = threadIdx.x; t < tot; t += kCgBlock) sh_red[t] = red[t];
        __syncthreads();
        if (threadIdx.x < 2 * KG) {
            double s = 0.0;
            for (int ww = 0; ww < A.W; ++ww) s += sh_red[ww * 2 * KG + threadIdx.x];
            sh_grp[threadIdx.x] = s;
        }
        __syncthreads();
    };

    // The matrix does not change during the solve: with one row per thread, keep the
    // first kCache entries of the row in registers.
    constexpr int kCache = 8;
    const bool cached = A.rows_per_thread == 1;
    int32_t cj[kCache];
    double cv[kCache];
    {
        const int64_t i = rb + threadIdx.x;
#pragma unroll
        for (int e = 0; e < kCache; ++e) {
            const bool in = cached && i < re && e < A.ell_w;
            cj[e] = in ? A.ecol[(int64_t)e * n + i] : 0;
            cv[e] = in ? A.eval[(int64_t)e * n + i] : 0.0;
        }
    }

    // sparse row i of C applied to y (row stride k, columns c0..c0+nc) -> acc
    auto spmv_row = [&](int64_t i, const double* y, int64_t ystride, double (&acc)[KG]) {
#pragma unroll
        for (int c = 0; c < KG; ++c) acc[c] = 0.0;
        for (int e = 0; e < A.ell_w; ++e) {
            const int64_t j = A.ecol[(int64_t)e * n + i];
            const double v = A.eval[(int64_t)e * n + i];
#pragma unroll
            for (int c = 0; c < KG; ++c)
                if (c < nc) acc[c] += v * y[j * ystride + c];
        }
    };

    double gam[KG], bb[KG], rr[KG], alpha[KG], beta[KG];
    bool done[KG];
    int its[KG];
#pragma unroll
    for (int c = 0; c < KG; ++c) {
        done[c] = (c >= nc);
        its[c] = 0;
        bb[c] = rr[c] = 0.0;
    }
    int total_it = 0;
    // Partial sums for the m-th barrier go to buffer m % 2: a buffer is rewritten only
    // after the next barrier, by which time every reader of it has arrived there.
    int bcount = 0;
    auto redbuf = [&]() { return redg + (int64_t)(bcount & 1) * A.W * 2 * KG; };
    constexpr int kMaxRestarts = 6;
    for (int cycle = 0; cycle <= kMaxRestarts; ++cycle) {
        // ---- R: r = b - C x (x = 0 on the first cycle), s = 0, p = 0; sums of r^2
        double loc[KG], dum[KG];
#pragma unroll
        for (int c = 0; c < KG; ++c) loc[c] = dum[c] = 0.0;
        for (int64_t i = rb + threadIdx.x; i < re; i += kCgBlock) {
            double cx[KG];
            if (cycle == 0) {
#pragma unroll
                for (int c = 0; c < KG; ++c) cx[c] = 0.0;
            } else {
                spmv_row(i, A.x + c0, k, cx);
            }
            double* zi = Z0 + i * zrow;
#pragma unroll
            for (int c = 0; c < KG; ++c) {
                if (c < nc) {
                    const int64_t id = i * k + c0 + c;
                    if (cycle == 0) A.x[id] = 0.0;
                    const double rv = A.b[id] - cx[c];
                    A.p[id] = 0.0;
                    zi[c0 + c] = rv;
                    zi[2 * k + c0 + c] = 0.0;
                    loc[c] += rv * rv;
                }
            }
        }
        block_sums2<KG>(loc, dum, sh_wave, sh_sum);
        if (threadIdx.x < 2 * KG) redbuf()[w * 2 * KG + threadIdx.x] = sh_sum[threadIdx.x];
        if (!group_barrier(gbar, w, A.W, A.flags, (unsigned)bcount + 1u)) return;
        group_sum(redbuf());
        ++bcount;
        bool all = true;
#pragma unroll
        for (int c = 0; c < KG; ++c) {
            rr[c] = sh_grp[c];
            if (cycle == 0) {
                bb[c] = rr[c];
                if (!(bb[c] > 0.0)) done[c] = true;
            }
            if (!done[c] && sqrt(rr[c] / bb[c]) <= A.rtol) done[c] = true;
            all = all && done[c];
        }
        __syncthreads();
        if (all || total_it >= A.maxiter) break;

        // ---- W: w = C r; gamma = (r, r), delta = (w, r)
        double ga[KG], de[KG];
#pragma unroll
        for (int c = 0; c < KG; ++c) ga[c] = de[c] = 0.0;
        for (int64_t i = rb + threadIdx.x; i < re; i += kCgBlock) {
            double acc[KG];
            spmv_row(i, Z0 + c0, zrow, acc);
            double* zi = Z0 + i * zrow;
#pragma unroll
            for (int c = 0; c < KG; ++c) {
                if (c < nc) {
                    const double rv = zi[c0 + c];
                    zi[k + c0 + c] = acc[c];
                    ga[c] += rv * rv;
                    de[c] += acc[c] * rv;
                }
            }
        }
        block_sums2<KG>(ga, de, sh_wave, sh_sum);
        if (threadIdx.x < 2 * KG) redbuf()[w * 2 * KG + threadIdx.x] = sh_sum[threadIdx.x];
        if (!group_barrier(gbar, w, A.W, A.flags, (unsigned)bcount + 1u)) return;
        group_sum(redbuf());
        ++bcount;
#pragma unroll
        for (int c = 0; c < KG; ++c) {
            gam[c] = sh_grp[c];
            beta[c] = 0.0;
            alpha[c] = done[c] ? 0.0 : gam[c] / sh_grp[KG + c];
        }
        __syncthreads();

        // ---- iterations until every open column meets rtol on the recursive residual
        for (int it = 0; total_it < A.maxiter; ++it) {
            ++total_it;
            const double* Zc = (it & 1) ? Z1 : Z0;
            double* Zn = (it & 1) ? Z0 : Z1;
#pragma unroll
            for (int c = 0; c < KG; ++c) ga[c] = de[c] = 0.0;
            for (int64_t i = rb + threadIdx.x; i < re; i += kCgBlock) {
                // w_{i+1} = C r_{i+1}, r_{i+1}(j) = r_i(j) - alpha (w_i(j) + beta s_{i-1}(j))
                double acc[KG];
#pragma unroll
                for (int c = 0; c < KG; ++c) acc[c] = 0.0;
                auto add_entry = [&](int64_t j, double v) {
                    const double* zj = Zc + j * zrow + c0;
#pragma unroll
                    for (int c = 0; c < KG; ++c)
                        if (c < nc) acc[c] += v * (zj[c] - alpha[c] * (zj[k + c] + beta[c] * zj[2 * k + c]));
                };
                int e0 = 0;
                if (cached) {
#pragma unroll
                    for (int e = 0; e < kCache; ++e)
                        if (e < A.ell_w) add_entry(cj[e], cv[e]);
                    e0 = kCache;
                }
                for (int e = e0; e < A.ell_w; ++e)
                    add_entry(A.ecol[(int64_t)e * n + i], A.eval[(int64_t)e * n + i]);
                const double* zi = Zc + i * zrow + c0;
                double* zo = Zn + i * zrow + c0;
#pragma unroll
                for (int c = 0; c < KG; ++c) {
                    if (c < nc) {
                        const int64_t id = i * k + c0 + c;
                        const double rv = zi[c], wv = zi[k + c], sv = zi[2 * k + c];
                        const double pn = rv + beta[c] * A.p[id];
                        const double sn = wv + beta[c] * sv;
                        A.p[id] = pn;
                        A.x[id] += alpha[c] * pn;
                        const double rn = rv - alpha[c] * sn;
                        zo[c] = rn;
                        zo[k + c] = acc[c];
                        zo[2 * k + c] = sn;
                        ga[c] += rn * rn;
                        de[c] += acc[c] * rn;
                    }
                }
            }
            block_sums2<KG>(ga, de, sh_wave, sh_sum);
            if (threadIdx.x < 2 * KG) redbuf()[w * 2 * KG + threadIdx.x] = sh_sum[threadIdx.x];
            if (!group_barrier(gbar, w, A.W, A.flags, (unsigned)bcount + 1u)) return;
            group_sum(redbuf());
            ++bcount;
            bool conv = true;
#pragma unroll
            for (int c = 0; c < KG; ++c) {
                if (!done[c] && alpha[c] != 0.0) {
                    const double gn = sh_grp[c], dn = sh_grp[KG + c];
                    its[c] = total_it;
                    rr[c] = gn;
                    if (sqrt(gn / bb[c]) <= A.rtol) {
                        alpha[c] = beta[c] = 0.0;       // frozen until verified
                    } else {
                        const double bn = gn / gam[c];
                        alpha[c] = gn / (dn - bn * gn / alpha[c]);
                        beta[c] = bn;
                        gam[c] = gn;
                        conv = false;
                    }
                }
            }
            __syncthreads();
            if (conv) break;
        }
        // the next cycle's R phase recomputes the true residual from x
    }
    if (w == 0 && threadIdx.x < nc) {
        const int c = threadIdx.x;
        A.iters[c0 + c] = its[c];
        A.relres[c0 + c] = bb[c] > 0.0 ? sqrt(rr[c] / bb[c]) : 0.0;
    }
}

// ------------------------------------------------------------------ CSR -> ELL

__global__ void k_csr_to_ell(int64_t n, const int32_t* __restrict__ off, const int32_t* __restrict__ col,
                             const double* __restrict__ val, int w, int32_t* __restrict__ ecol,
                             double* __restrict__ eval)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t b = off[i], len = off[i + 1] - b;
    for (int e = 0; e < w; ++e) {
        const bool in = e < len;
        ecol[(int64_t)e * n + i] = in ? col[b + e] : (int32_t)i;
        eval[(int64_t)e * n + i] = in ? val[b + e] : 0.0;
    }
}

hipError_t launch_csr_to_ell(int64_t n, const int32_t* off, const int32_t* col, const double* val,
                             int w, int32_t* ecol, double* eval, hipStream_t s)
{
    hipLaunchKernelGGL(k_csr_to_ell, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, off, col, val, w, ecol, eval);
    return hipGetLastError();
}

// ------------------------------------------------------------------ launch

namespace {

struct CgShape {
    int kg, ngroups;
};

CgShape cg_shape(int k)
{
    CgShape s;
    s.ngroups = (k + kMaxGroupCols - 1) / kMaxGroupCols;
    s.kg = (k + s.ngroups - 1) / s.ngroups;
    return s;
}

// Rows per thread and workgroups per group: one row per thread while the group fits in
// kMaxW workgroups and the whole grid stays co-resident (a cooperative launch needs it).
template <int KG>
hipError_t launch_cg_k(CgArgs a, hipStream_t s)
{
    const void* fn = (const void*)k_cg<KG>;
    int per_cu = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kCgBlock, 0);
    if (e != hipSuccess) return e;
    const int64_t capacity = (int64_t)per_cu * device_info().num_cu;
    const int64_t wmax = std::min<int64_t>(kMaxW, capacity / a.ngroups);
    if (wmax < 1) return hipErrorCooperativeLaunchTooLarge;
    const int64_t wg_rows = (a.n + kCgBlock - 1) / kCgBlock;
    a.rows_per_thread = (int)((wg_rows + wmax - 1) / wmax);
    a.W = (int)((a.n + (int64_t)kCgBlock * a.rows_per_thread - 1) / ((int64_t)kCgBlock * a.rows_per_thread));
    if (a.W < 1) a.W = 1;
    void* params[] = {&a};
    return hipLaunchCooperativeKernel(fn, dim3((unsigned)(a.ngroups * a.W)), dim3(kCgBlock), params, 0, s);
}

}  // namespace

size_t cg_red_doubles(int k)
{
    (void)k;
    return (size_t)kMaxGroups * 2 * kMaxW * 2 * kMaxGroupCols;
}

size_t cg_bar_words(int k)
{
    (void)k;
    return (size_t)kMaxGroups * kBarWordsPerGroup;
}

size_t cg_state_doubles(int64_t n, int k) { return (size_t)2 * n * 3 * k; }

hipError_t launch_cg(int64_t n, const int32_t* ecol, const double* eval, int ell_w,
                     const double* b, double* x, int k, double rtol, int maxiter,
                     const CgWork& w, hipStream_t s)
{
    const CgShape sh = cg_shape(k);
    if (sh.ngroups > kMaxGroups || sh.kg > kMaxGroupCols) return hipErrorInvalidValue;
    hipError_t e = hipMemsetAsync(w.bar, 0, cg_bar_words(k) * sizeof(unsigned), s);
    if (e != hipSuccess) return e;
    CgArgs a;
    a.n = n; a.ell_w = ell_w; a.ecol = ecol; a.eval = eval; a.b = b; a.x = x;
    a.Z = w.Z; a.p = w.p; a.red = w.red; a.bar = w.bar;
    a.iters = w.iters; a.relres = w.relres; a.flags = w.flags;
    a.rtol = rtol; a.maxiter = maxiter; a.k = k; a.ngroups = sh.ngroups; a.W = 1;
    a.rows_per_thread = 1;
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
