// Static obstacle potential (Sec. 7.3.2) on the GPU, FP64 pair terms: one thread per surface
// face T, the obstacle's faces streamed through LDS in tiles of kTileJ (every lane reads the
// same obstacle face).  Per pair, with d = X_T - X_O(S) and r2 = |d|^2:
//   w = a_O(S) r2^(-p/2),  phi(T) += w,  dphi/dX_T += -p w d / r2.
// Sums run over the obstacle in a fixed order, so results are reproducible.
#include "tp_obstacle.h"
#include "tp_tree.h"

namespace tp {

namespace {

inline unsigned nblk(int64_t n, int b = 256) { return (unsigned)((n + b - 1) / b); }

__global__ void k_obs_faces(const double* __restrict__ Vo, const int32_t* __restrict__ Fo, int64_t nFo,
                            int64_t cap_o, double4* __restrict__ xo)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= cap_o) return;
    if (t >= nFo) {   // padding: zero area far away (its terms are 0 * tiny)
        xo[t] = make_double4(1e15, 1e15, 1e15, 0.0);
        return;
    }
    const double* a = Vo + 3 * (int64_t)Fo[3 * t];
    const double* b = Vo + 3 * (int64_t)Fo[3 * t + 1];
    const double* c = Vo + 3 * (int64_t)Fo[3 * t + 2];
    const double e1[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
    const double e2[3] = {c[0] - a[0], c[1] - a[1], c[2] - a[2]};
    const double cr[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2], e1[0] * e2[1] - e1[1] * e2[0]};
    xo[t] = make_double4((a[0] + b[0] + c[0]) / 3.0, (a[1] + b[1] + c[1]) / 3.0, (a[2] + b[2] + c[2]) / 3.0,
                         0.5 * sqrt(cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2]));
}

template <bool P6>
__global__ __launch_bounds__(kBlock) void k_obs_pairs(const double4* __restrict__ dx, int64_t nF,
                                                      const double4* __restrict__ xo, int64_t cap_o, double p,
                                                      double* __restrict__ e, double* __restrict__ g, int64_t gs)
{
    __shared__ double4 s_o[kTileJ];
    const int64_t T = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const double4 x = dx[T < nF ? T : 0];
    double phi = 0.0, g0 = 0.0, g1 = 0.0, g2 = 0.0;
    for (int64_t j0 = 0; j0 < cap_o; j0 += kTileJ) {
        __syncthreads();
        for (int q = threadIdx.x; q < kTileJ; q += kBlock) s_o[q] = xo[j0 + q];
        __syncthreads();
        for (int q = 0; q < kTileJ; ++q) {
            const double4 o = s_o[q];
            const double d0 = x.x - o.x, d1 = x.y - o.y, d2 = x.z - o.z;
            const double r2 = d0 * d0 + d1 * d1 + d2 * d2;
            const double inv = 1.0 / r2;
            const double w = o.w * (P6 ? inv * inv * inv : pow(r2, -0.5 * p));
            phi += w;
            const double c = -p * w * inv;
            g0 += c * d0;
            g1 += c * d1;
            g2 += c * d2;
        }
    }
    if (T >= nF) return;
    e[T] = x.w * phi;
    g[T] = x.w * g0;
    g[gs + T] = x.w * g1;
    g[2 * gs + T] = x.w * g2;
    g[3 * gs + T] = 0.0;
    g[4 * gs + T] = 0.0;
    g[5 * gs + T] = 0.0;
    g[6 * gs + T] = phi;
}

// Barnes-Hut form (params.theta > 0): the tree of launch_bh_build over the obstacle's faces,
// one thread per surface face, the lanes of a wave walking it together (wave_walk).  The
// potential is evaluated at the barycenter X_T, a point, so node I is admissible when
// r_I^2 < theta^2 dist(X_T, box_I)^2 (decided in FP64 without fused multiply-adds, so the
// interaction lists are a function of the meshes alone) and then contributes
// a_I |X_I - X_T|^-p; a leaf that is not admissible contributes its faces one by one.  Each
// thread sums its own terms in traversal order; the term counts are summed per wave and
// added with one integer atomic per wave.
struct ObsTreeArgs {
    const double4* dx;        // surface face data (X_T, a_T)
    int64_t nF;
    const double4* xo;        // obstacle face data (X_O, a_O), caller's obstacle numbering
    const int32_t* order;     // sorted position -> obstacle face
    const double* na;
    const double* nX;
    const double* nlo;
    const double* nhi;
    const double* nr2;
    int64_t nFo, P;
    int leaf;
    double theta2, p;
    double* e;
    double* g;
    int64_t gs;
    unsigned long long* counts;
};

__device__ __forceinline__ bool point_admissible(const ObsTreeArgs& A, const double4& x, int64_t node)
{
#pragma clang fp contract(off)
    double d2 = 0.0;
    const double xs[3] = {x.x, x.y, x.z};
    for (int m = 0; m < 3; ++m) {
        const double g1 = A.nlo[3 * node + m] - xs[m];
        const double g2 = xs[m] - A.nhi[3 * node + m];
        double gm = g1 > g2 ? g1 : g2;
        gm = gm < 0.0 ? 0.0 : gm;
        d2 = d2 + gm * gm;
    }
    return A.nr2[node] < A.theta2 * d2;
}

template <bool P6>
__global__ __launch_bounds__(256) void k_obs_bh(ObsTreeArgs A)
{
    const int64_t T = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool live = T < A.nF;                 // every lane walks with its wave
    const double4 x = A.dx[live ? T : 0];
    double phi = 0.0, g0 = 0.0, g1 = 0.0, g2 = 0.0;
    unsigned long long nfar = 0, nnear = 0;
    auto visit = [&](double yx, double yy, double yz, double w) {
        const double d0 = x.x - yx, d1 = x.y - yy, d2 = x.z - yz;
        const double r2 = d0 * d0 + d1 * d1 + d2 * d2;
        const double inv = 1.0 / r2;
        const double t = w * (P6 ? inv * inv * inv : pow(r2, -0.5 * A.p));
        phi += t;
        const double c = -A.p * t * inv;
        g0 += c * d0;
        g1 += c * d1;
        g2 += c * d2;
    };
    wave_walk(
        A.na, A.P, live, [&](int node) { return point_admissible(A, x, node); },
        [&](int node) {
            visit(A.nX[3 * node], A.nX[3 * node + 1], A.nX[3 * node + 2], A.na[node]);
            ++nfar;
        },
        [&](int node) {
            const int64_t l = node - A.P;
            const int64_t q1 = min((l + 1) * (int64_t)A.leaf, A.nFo);
            for (int64_t q = l * A.leaf; q < q1; ++q) {
                const double4 o = A.xo[A.order[q]];
                visit(o.x, o.y, o.z, o.w);
                ++nnear;
            }
        });
    wave_count_terms(A.counts, nfar, nnear);
    if (!live) return;
    const int64_t gs = A.gs;
    A.e[T] = x.w * phi;
    A.g[T] = x.w * g0;
    A.g[gs + T] = x.w * g1;
    A.g[2 * gs + T] = x.w * g2;
    A.g[3 * gs + T] = 0.0;
    A.g[4 * gs + T] = 0.0;
    A.g[5 * gs + T] = 0.0;
    A.g[6 * gs + T] = phi;
}

__global__ void k_implicit(const double4* __restrict__ dx, int64_t nF, ImplicitSet set, double* __restrict__ e,
                           double* __restrict__ g, int64_t gs)
{
    const int64_t T = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (T >= nF) return;
    const double4 x = dx[T];
    double phi = 0.0, g0 = 0.0, g1 = 0.0, g2 = 0.0;
    for (int k = 0; k < set.n; ++k) {
        double d, n0, n1, n2;   // signed distance and its gradient
        if (set.kind[k] == 0) {
            n0 = set.q[k][0]; n1 = set.q[k][1]; n2 = set.q[k][2];
            d = n0 * x.x + n1 * x.y + n2 * x.z - set.c[k];
        } else {
            const double r0 = x.x - set.q[k][0], r1 = x.y - set.q[k][1], r2 = x.z - set.q[k][2];
            const double r = sqrt(r0 * r0 + r1 * r1 + r2 * r2);
            n0 = r0 / r; n1 = r1 / r; n2 = r2 / r;
            d = r - set.c[k];
        }
        const double p = set.p[k], w = set.w[k];
        double f, df;   // potential and its derivative in d
        if (set.attract[k]) {
            const double ad = fabs(d);
            f = pow(ad, p);
            df = ad > 0.0 ? p * f / d : 0.0;
        } else if (d > 0.0) {
            f = pow(d, -p);
            df = -p * f / d;
        } else {
            // on or inside the obstacle: the potential is infinite whatever p is (for an
            // even integer p, pow(d, -p) would be finite on the far side of the barrier,
            // and for an odd one negative), so the line search rejects such a step
            f = INFINITY;
            df = -INFINITY;
        }
        phi += w * f;
        g0 += w * df * n0;
        g1 += w * df * n1;
        g2 += w * df * n2;
    }
    e[T] = x.w * phi;
    g[T] = x.w * g0;
    g[gs + T] = x.w * g1;
    g[2 * gs + T] = x.w * g2;
    g[3 * gs + T] = 0.0;
    g[4 * gs + T] = 0.0;
    g[5 * gs + T] = 0.0;
    g[6 * gs + T] = phi;
}

__global__ void k_vertex_area(int64_t nV, const int32_t* __restrict__ vf_off, const int32_t* __restrict__ vf_idx,
                              const double4* __restrict__ dx, double* __restrict__ out)
{
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= nV) return;
    double a = 0.0;
    for (int32_t q = vf_off[v]; q < vf_off[v + 1]; ++q) a += dx[vf_idx[q] / 3].w / 3.0;
    out[v] = a;
}

__global__ void k_add_translation(double* __restrict__ x, const int32_t* __restrict__ label,
                                  const double* __restrict__ t, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= 3 * n) return;
    x[i] += t[3 * (int64_t)label[i / 3] + i % 3];
}

}  // namespace

hipError_t launch_implicit(const double4* dx, int64_t nF, const ImplicitSet& set, double* e, double* g, int64_t gs,
                           hipStream_t s)
{
    if (set.n < 1 || set.n > kMaxImplicit || gs < nF) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_implicit, dim3(nblk(nF)), dim3(256), 0, s, dx, nF, set, e, g, gs);
    return hipGetLastError();
}

hipError_t launch_vertex_area(int64_t nV, const int32_t* vf_off, const int32_t* vf_idx, const double4* dx,
                              double* out, hipStream_t s)
{
    hipLaunchKernelGGL(k_vertex_area, dim3(nblk(nV)), dim3(256), 0, s, nV, vf_off, vf_idx, dx, out);
    return hipGetLastError();
}

hipError_t launch_add_translation(double* x, const int32_t* label, const double* t, int64_t n, hipStream_t s)
{
    hipLaunchKernelGGL(k_add_translation, dim3(nblk(3 * n)), dim3(256), 0, s, x, label, t, n);
    return hipGetLastError();
}

int64_t obstacle_capacity(int64_t nFo) { return (std::max<int64_t>(nFo, 1) + kTileJ - 1) / kTileJ * kTileJ; }

hipError_t launch_obstacle_faces(const double* Vo, const int32_t* Fo, int64_t nFo, int64_t cap_o, double4* xo,
                                 hipStream_t s)
{
    if (cap_o % kTileJ != 0 || cap_o < nFo) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_obs_faces, dim3(nblk(cap_o)), dim3(256), 0, s, Vo, Fo, nFo, cap_o, xo);
    return hipGetLastError();
}

hipError_t launch_obstacle_pairs(const double4* dx, int64_t nF, const double4* xo, int64_t cap_o, double p,
                                 double* e, double* g, int64_t gs, hipStream_t s)
{
    if (cap_o % kTileJ != 0 || nF < 1 || gs < nF) return hipErrorInvalidValue;
    if (p == 6.0)
        hipLaunchKernelGGL(k_obs_pairs<true>, dim3(nblk(nF, kBlock)), dim3(kBlock), 0, s, dx, nF, xo, cap_o, p, e, g, gs);
    else
        hipLaunchKernelGGL(k_obs_pairs<false>, dim3(nblk(nF, kBlock)), dim3(kBlock), 0, s, dx, nF, xo, cap_o, p, e, g, gs);
    return hipGetLastError();
}

hipError_t launch_obstacle_bh(const double4* dx, int64_t nF, const double4* xo, const BhBuffers& tree, int64_t nFo,
                              int leaf, double theta, double p, double* e, double* g, int64_t gs,
                              unsigned long long* counts, hipStream_t s)
{
    if (nF < 1 || nFo < 1 || gs < nF || leaf < 1) return hipErrorInvalidValue;
    int64_t P = 0;
    (void)bh_node_count(nFo, leaf, &P);
    hipError_t err = hipMemsetAsync(counts, 0, 2 * sizeof(unsigned long long), s);
    if (err != hipSuccess) return err;
    ObsTreeArgs A;
    A.dx = dx; A.nF = nF; A.xo = xo; A.order = tree.order; A.na = tree.na; A.nX = tree.nX; A.nlo = tree.nlo;
    A.nhi = tree.nhi; A.nr2 = tree.nr2; A.nFo = nFo; A.P = P; A.leaf = leaf; A.theta2 = theta * theta; A.p = p;
    A.e = e; A.g = g; A.gs = gs; A.counts = counts;
    if (p == 6.0) hipLaunchKernelGGL(k_obs_bh<true>, dim3(nblk(nF)), dim3(256), 0, s, A);
    else hipLaunchKernelGGL(k_obs_bh<false>, dim3(nblk(nF)), dim3(256), 0, s, A);
    return hipGetLastError();
}

}  // namespace tp
