// Barnes-Hut approximation of the energy and its differential (Sec. 4) on gfx950.
//
// Tree.  Faces are sorted by the 30-bit Morton code of their barycenters (10 bits per
// coordinate, quantized on the bounding box of all barycenters), ties by the caller's face
// number (faces are stored internally in the Morton order of the first mesh).  Leaves hold `leaf` consecutive sorted
// faces and the internal nodes form a perfect binary tree over the leaves in heap order
// (node 1 is the root, node i has children 2i and 2i + 1, the leaves are nodes
// P .. 2P - 1).  The tree is therefore fixed by the sort alone: no pointer chasing, and
// the traversal needs no stack (the next node after a subtree follows from the heap
// index).  Node quantities are built level by level: a_I, sum a_T X_T, the bounding box of
// the faces' vertices, X_I and r_I^2 (largest squared distance from X_I to a box corner).
// The geometric quantities that decide admissibility are formed in FP64 without fused
// multiply-adds, in a fixed order, so the interaction lists are a function of the mesh.
//
// Admissibility: node I is admissible for face S when max(r_S^2, r_I^2) < theta^2 dist^2
// (r_S: largest distance from X_S to a corner of S; dist: distance between the box of S's
// vertices and the box of I).
//
// Traversal.  One thread per face, threads in Morton order, and the 64 lanes of a wave walk
// the tree together (wave_walk): the wave visits the union of its lanes' lists in
// depth-first order, each lane taking its own terms in the order of its own walk, and every
// lane reads the same node at the same time.  An admissible node adds K(X_S, N_S; X_I)
// a_S a_I, a leaf that is not admissible adds the exact terms of its faces T != S, other
// nodes are opened.  The
// differential is that of E_BH with the lists held fixed: the face S side is summed per
// thread; the target side (dX, da of a face T or a node I) is summed across the wave and
// added with device-scope atomics, one set per wave and target; node derivatives then
// reach their member faces through X_I = sum a_T X_T / a_I and a_I = sum a_T, walking up
// each face's ancestors.  The atomic sums make the last bits
// of dE depend on scheduling; E itself is summed per face in a fixed order.
#include "tp_internal.h"
#include "tp_tree.h"

#include <hipcub/hipcub.hpp>

#include <algorithm>

namespace tp {

namespace {

#pragma clang fp contract(off)

__device__ __forceinline__ uint32_t spread10(uint32_t v)
{
    uint32_t out = 0;
    for (int b = 0; b < 10; ++b) out |= ((v >> b) & 1u) << (3 * b);
    return out;
}

__device__ __forceinline__ uint32_t quant10(double x, double lo, double hi)
{
    if (!(hi > lo)) return 0u;
    double t = floor(1024.0 * ((x - lo) / (hi - lo)));
    t = t < 0.0 ? 0.0 : (t > 1023.0 ? 1023.0 : t);
    return (uint32_t)t;
}

// Face boxes (of the three vertices) and r_S^2.
__global__ void k_bh_faceprep(const double* __restrict__ V, const int32_t* __restrict__ F, int64_t nF,
                              const double4* __restrict__ dx, double* __restrict__ flo,
                              double* __restrict__ fhi, double* __restrict__ fr2)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= nF) return;
    const double4 X = dx[s];
    const double xs[3] = {X.x, X.y, X.z};
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    double best = 0.0;
    for (int c = 0; c < 3; ++c) {
        const double* v = V + 3 * (int64_t)F[3 * s + c];
        double d2 = 0.0;
        for (int m = 0; m < 3; ++m) {
            lo[m] = v[m] < lo[m] ? v[m] : lo[m];
            hi[m] = v[m] > hi[m] ? v[m] : hi[m];
            const double dm = v[m] - xs[m];
            d2 = d2 + dm * dm;
        }
        best = d2 > best ? d2 : best;
    }
    for (int m = 0; m < 3; ++m) {
        flo[3 * s + m] = lo[m];
        fhi[3 * s + m] = hi[m];
    }
    fr2[s] = best;
}

// Bounding box of the barycenters (one workgroup; min and max do not depend on order).
__global__ __launch_bounds__(1024) void k_bh_bbox(const double4* __restrict__ dx, int64_t nF,
                                                  double* __restrict__ box)
{
    __shared__ double sh[6][1024];
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int64_t s = threadIdx.x; s < nF; s += blockDim.x) {
        const double4 X = dx[s];
        const double x[3] = {X.x, X.y, X.z};
        for (int m = 0; m < 3; ++m) {
            lo[m] = x[m] < lo[m] ? x[m] : lo[m];
            hi[m] = x[m] > hi[m] ? x[m] : hi[m];
        }
    }
    for (int m = 0; m < 3; ++m) {
        sh[m][threadIdx.x] = lo[m];
        sh[3 + m][threadIdx.x] = hi[m];
    }
    __syncthreads();
    for (int w = 512; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int m = 0; m < 3; ++m) {
                const double a = sh[m][threadIdx.x + w], b = sh[3 + m][threadIdx.x + w];
                sh[m][threadIdx.x] = a < sh[m][threadIdx.x] ? a : sh[m][threadIdx.x];
                sh[3 + m][threadIdx.x] = b > sh[3 + m][threadIdx.x] ? b : sh[3 + m][threadIdx.x];
            }
        __syncthreads();
    }
    if (threadIdx.x < 6) box[threadIdx.x] = sh[threadIdx.x][0];
}

// Keys (Morton code << 32 | caller's face number) and the internal face index as value;
// the caller's numbers make the order independent of how faces are stored.
__global__ void k_bh_keys(const double4* __restrict__ dx, int64_t nF, const double* __restrict__ box,
                          const int32_t* __restrict__ orig, uint64_t* __restrict__ keys,
                          int32_t* __restrict__ idx)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= nF) return;
    const double4 X = dx[s];
    const uint32_t code = (spread10(quant10(X.x, box[0], box[3])) << 2) |
                          (spread10(quant10(X.y, box[1], box[4])) << 1) | spread10(quant10(X.z, box[2], box[5]));
    keys[s] = ((uint64_t)code << 32) | (uint64_t)(uint32_t)(orig ? orig[s] : (int32_t)s);
    idx[s] = (int32_t)s;
}

__global__ void k_bh_pos(const int32_t* __restrict__ order, int64_t nF, int32_t* __restrict__ pos)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= nF) return;
    pos[order[p]] = (int32_t)p;
}

// Leaf nodes P + l: sums over the member faces in sorted order.
__global__ void k_bh_leaves(int64_t nF, int leaf, int64_t P, const int32_t* __restrict__ order,
                            const double4* __restrict__ dx, const double* __restrict__ flo,
                            const double* __restrict__ fhi, double* __restrict__ na,
                            double* __restrict__ nsx, double* __restrict__ nlo, double* __restrict__ nhi)
{
    const int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= P) return;
    const int64_t node = P + l;
    double a = 0.0, sx[3] = {0.0, 0.0, 0.0};
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int64_t p = l * leaf; p < (l + 1) * leaf && p < nF; ++p) {
        const int32_t s = order[p];
        const double4 X = dx[s];
        const double x[3] = {X.x, X.y, X.z};
        a = a + X.w;
        for (int m = 0; m < 3; ++m) {
            sx[m] = sx[m] + X.w * x[m];
            lo[m] = flo[3 * s + m] < lo[m] ? flo[3 * s + m] : lo[m];
            hi[m] = fhi[3 * s + m] > hi[m] ? fhi[3 * s + m] : hi[m];
        }
    }
    na[node] = a;
    for (int m = 0; m < 3; ++m) {
        nsx[3 * node + m] = sx[m];
        nlo[3 * node + m] = lo[m];
        nhi[3 * node + m] = hi[m];
    }
}

__device__ __forceinline__ void bh_node_finish(int64_t node, const double* __restrict__ na,
                                               const double* __restrict__ nsx, const double* __restrict__ nlo,
                                               const double* __restrict__ nhi, double* __restrict__ nX,
                                               double* __restrict__ nr2)
{
    const double a = na[node];
    if (!(a > 0.0)) {
        nr2[node] = 0.0;
        for (int m = 0; m < 3; ++m) nX[3 * node + m] = 0.0;
        return;
    }
    double r2 = 0.0;
    for (int m = 0; m < 3; ++m) {
        const double x = nsx[3 * node + m] / a;
        nX[3 * node + m] = x;
        const double u = x - nlo[3 * node + m], v = nhi[3 * node + m] - x;
        const double w = u > v ? u : v;
        r2 = r2 + w * w;
    }
    nr2[node] = r2;
}

// Internal nodes level by level (children before parents) in one workgroup, then the
// node barycenters and radii of all nodes.
__global__ __launch_bounds__(1024) void k_bh_levels(int64_t P, double* __restrict__ na, double* __restrict__ nsx,
                                                    double* __restrict__ nlo, double* __restrict__ nhi,
                                                    double* __restrict__ nX, double* __restrict__ nr2)
{
    for (int64_t n0 = P / 2; n0 >= 1; n0 /= 2) {
        for (int64_t node = n0 + threadIdx.x; node < 2 * n0; node += blockDim.x) {
            const int64_t L = 2 * node, R = 2 * node + 1;
            na[node] = na[L] + na[R];
            for (int m = 0; m < 3; ++m) {
                nsx[3 * node + m] = nsx[3 * L + m] + nsx[3 * R + m];
                nlo[3 * node + m] = nlo[3 * L + m] < nlo[3 * R + m] ? nlo[3 * L + m] : nlo[3 * R + m];
                nhi[3 * node + m] = nhi[3 * L + m] > nhi[3 * R + m] ? nhi[3 * L + m] : nhi[3 * R + m];
            }
        }
        __syncthreads();
    }
    for (int64_t node = 1 + threadIdx.x; node < 2 * P; node += blockDim.x)
        bh_node_finish(node, na, nsx, nlo, nhi, nX, nr2);
}

#pragma clang fp contract(fast)

struct BhArgs {
    int64_t nF, P;
    int leaf;
    double theta2;
    double alpha, beta;
    const int32_t* order;
    const double4* dx;
    const double4* dn;
    const double* flo;
    const double* fhi;
    const double* fr2;
    const double* na;
    const double* nX;
    const double* nlo;
    const double* nhi;
    const double* nr2;
    double* gS;           // [7][nF] face-side sums (gradient only)
    double* eS;           // [nF] energy rows
    double* accF;         // [4][nF] target-side sums of faces
    double* accN;         // [4][2P] target-side sums of nodes
    unsigned long long* counts;   // far, near
};

__device__ __forceinline__ bool admissible(const BhArgs& A, const double (&slo)[3], const double (&shi)[3],
                                           double sr2, int64_t node)
{
#pragma clang fp contract(off)
    double d2 = 0.0;
    for (int m = 0; m < 3; ++m) {
        const double g1 = A.nlo[3 * node + m] - shi[m];
        const double g2 = slo[m] - A.nhi[3 * node + m];
        double g = g1 > g2 ? g1 : g2;
        g = g < 0.0 ? 0.0 : g;
        d2 = d2 + g * g;
    }
    const double nr = A.nr2[node];
    const double r2 = sr2 > nr ? sr2 : nr;
    return r2 < A.theta2 * d2;
}

// Kernel and its derivatives for one target (R = float or double pair terms).
template <class R, bool GEN>
__device__ __forceinline__ void term(const double (&xs)[3], const double (&ns)[3], const double* y,
                                     const BhArgs& A, R& K, R (&dKdd)[3], R (&dKdN)[3])
{
    R d[3], n[3];
    for (int m = 0; m < 3; ++m) {
        d[m] = (R)(xs[m] - y[m]);
        n[m] = (R)ns[m];
    }
    const R r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
    const R q = n[0] * d[0] + n[1] * d[1] + n[2] * d[2];
    const R inv = (R)1 / r2;
    R Kqr;
    if (!GEN) {
        const R u = q * inv, u2 = u * u, u4 = u2 * u2;
        K = u4 * u2;           // |q|^6 r2^-6
        Kqr = u4 * u;          // sgn(q) |q|^5 r2^-5 = K r2 / q
    } else {
        const R aq = q < (R)0 ? -q : q;
        if (aq == (R)0) {
            K = (R)0;
            Kqr = (R)0;
        } else {
            Kqr = (R)pow((double)aq, A.alpha - 1.0) * (R)pow((double)r2, 1.0 - 0.5 * A.beta);
            Kqr = q < (R)0 ? -Kqr : Kqr;
            K = Kqr * q * inv;
        }
    }
    const R c1 = (R)A.alpha * Kqr * inv, c2 = (R)A.beta * K * inv;
    for (int m = 0; m < 3; ++m) {
        dKdd[m] = c1 * n[m] - c2 * d[m];
        dKdN[m] = c1 * d[m];
    }
}

template <class R, bool GEN, bool GRAD>
__global__ __launch_bounds__(256) void k_bh_traverse(BhArgs A)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool live = p < A.nF;                 // every lane walks with its wave
    const int32_t s = A.order[live ? p : 0];
    const double4 X = A.dx[s], Nn = A.dn[s];
    const double xs[3] = {X.x, X.y, X.z}, ns[3] = {Nn.x, Nn.y, Nn.z};
    const double aS = X.w;
    double slo[3], shi[3];
    for (int m = 0; m < 3; ++m) {
        slo[m] = A.flo[3 * s + m];
        shi[m] = A.fhi[3 * s + m];
    }
    const double sr2 = A.fr2[s];
    double gX[3] = {0, 0, 0}, gN[3] = {0, 0, 0}, ga = 0.0, e = 0.0;
    unsigned long long nfar = 0, nnear = 0;

    // one term of this lane with target (y, w): face-side sums here, target-side parts in tg
    auto visit = [&](const double* y, double w, double (&tg)[4]) {
        R K, dKdd[3], dKdN[3];
        term<R, GEN>(xs, ns, y, A, K, dKdd, dKdN);
        const double Kd = (double)K;
        e += aS * w * Kd;
        if (GRAD) {
            const double f = aS * w;
            for (int m = 0; m < 3; ++m) {
                const double gd = f * (double)dKdd[m];
                gX[m] += gd;
                gN[m] += f * (double)dKdN[m];
                tg[m] = -gd;
            }
            ga += w * Kd;
            tg[3] = aS * Kd;
        }
    };
    // the target-side parts of the wave's lanes are summed across the wave first, so each
    // target receives one set of atomic additions per wave
    auto push = [&](const double (&tg)[4], double* acc, int64_t stride) {
        for (int m = 0; m < 4; ++m) {
            const double v = wave_sum(tg[m]);
            if ((threadIdx.x & 63) == 0) unsafeAtomicAdd(acc + m * stride, v);
        }
    };

    wave_walk_act(
        A.na, A.P, live, [&](int node) { return admissible(A, slo, shi, sr2, node); },
        [&](int node, int took) {
            if (__ballot(took == 1) != 0ull) {
                double tg[4] = {0.0, 0.0, 0.0, 0.0};
                if (took == 1) {
                    visit(A.nX + 3 * (int64_t)node, A.na[node], tg);
                    ++nfar;
                }
                if (GRAD) push(tg, A.accN + node, 2 * A.P);
            }
            if (__ballot(took == 2) != 0ull) {
                const int64_t l = node - A.P;
                const int64_t p1 = min((l + 1) * (int64_t)A.leaf, A.nF);
                for (int64_t q = l * A.leaf; q < p1; ++q) {
                    const int32_t t = A.order[q];
                    double tg[4] = {0.0, 0.0, 0.0, 0.0};
                    if (took == 2 && t != s) {
                        const double4 Y = A.dx[t];
                        const double y[3] = {Y.x, Y.y, Y.z};
                        visit(y, Y.w, tg);
                        ++nnear;
                    }
                    if (GRAD) push(tg, A.accF + t, A.nF);
                }
            }
        });
    wave_count_terms(A.counts, nfar, nnear);
    if (!live) return;
    A.eS[s] = e;
    if (GRAD) {
        for (int m = 0; m < 3; ++m) {
            A.gS[m * A.nF + s] = gX[m];
            A.gS[(3 + m) * A.nF + s] = gN[m];
        }
        A.gS[6 * A.nF + s] = ga;
    }
}

// Per-face partial derivatives: face side + target side + the node terms of every
// ancestor, written as gface[m * gstride + t] (dE/dX, dE/dN, dE/da).
__global__ void k_bh_assemble(int64_t nF, int leaf, int64_t P, const int32_t* __restrict__ pos,
                              const double4* __restrict__ dx, const double* __restrict__ na,
                              const double* __restrict__ nX, const double* __restrict__ gS,
                              const double* __restrict__ accF, const double* __restrict__ accN,
                              double* __restrict__ gface, int64_t gstride)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nF) return;
    const double4 X = dx[t];
    const double xt[3] = {X.x, X.y, X.z};
    double gx[3], ga = gS[6 * nF + t] + accF[3 * nF + t];
    for (int m = 0; m < 3; ++m) gx[m] = gS[m * nF + t] + accF[m * nF + t];
    const int64_t M = 2 * P;
    for (int64_t node = P + pos[t] / leaf; node >= 1; node >>= 1) {
        const double a = na[node];
        if (!(a > 0.0)) continue;
        double proj = 0.0;
        for (int m = 0; m < 3; ++m) {
            const double g = accN[m * M + node];
            gx[m] += (X.w / a) * g;
            proj += (xt[m] - nX[3 * node + m]) * g;
        }
        ga += accN[3 * M + node] + proj / a;
    }
    for (int m = 0; m < 3; ++m) {
        gface[m * gstride + t] = gx[m];
        gface[(3 + m) * gstride + t] = gS[(3 + m) * nF + t];
    }
    gface[6 * gstride + t] = ga;
}

// ---------------------------------------------------------------- fractional apply
//
// The kernel matrix of the fractional operator (Sec. 5.1.1) with the same tree, the same
// admissibility and the same traversal as the energy: for face S an admissible node I adds
// k(X_S, X_I) (a_I ubar_S - m_I), m_I = sum_{T in I} a_T ubar_T (the node's moments), a leaf
// that is not admissible adds k(X_S, X_T) a_T (ubar_S - ubar_T) for its faces T != S, with
// k = |d|^-(2 sigma + 2).  Only the face S side is summed, so there are no atomics and
// the result is deterministic.  z(S) (without the factor a_S) goes to z[c * zstride + S],
// the layout of the direct kernel's reduced sums.
//
// Rows of face averages (ub), node moments (nm) and far-field values are KP wide, KP = the
// column count rounded up to 4 (the padding holds zeros), and are read as 4-wide vectors,
// so a row costs one memory round trip; the kernels are instantiated for KP = 4, 8, 12.

template <class UB> struct Vec4Of;
template <> struct Vec4Of<float> { using type = float4; };
template <> struct Vec4Of<double> { using type = double4; };

// out[0 .. KP) = row[0 .. KP) (16- or 32-byte aligned)
template <int KP, class T>
__device__ __forceinline__ void load_row(const T* __restrict__ row, double (&out)[KP])
{
    using V = typename Vec4Of<T>::type;
#pragma unroll
    for (int h = 0; h < KP / 4; ++h) {
        const V v = reinterpret_cast<const V*>(row)[h];
        out[4 * h] = (double)v.x;
        out[4 * h + 1] = (double)v.y;
        out[4 * h + 2] = (double)v.z;
        out[4 * h + 3] = (double)v.w;
    }
}

// Node moments [2P][KP], leaves first (member faces in sorted order), then level by level.
template <class UB, int KP>
__global__ void k_bh_moment_leaves(int64_t nF, int leaf, int64_t P, const int32_t* __restrict__ order,
                                   const double4* __restrict__ dx, const UB* __restrict__ ub,
                                   double* __restrict__ nm)
{
    const int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= P) return;
    double acc[KP];
#pragma unroll
    for (int c = 0; c < KP; ++c) acc[c] = 0.0;
    for (int64_t p = l * leaf; p < (l + 1) * leaf && p < nF; ++p) {
        const int32_t t = order[p];
        const double a = dx[t].w;
        double u[KP];
        load_row<KP>(ub + (int64_t)t * KP, u);
#pragma unroll
        for (int c = 0; c < KP; ++c) acc[c] = acc[c] + a * u[c];
    }
#pragma unroll
    for (int c = 0; c < KP; ++c) nm[(P + l) * KP + c] = acc[c];
}

__global__ __launch_bounds__(1024) void k_bh_moment_levels(int64_t P, int kp, double* __restrict__ nm)
{
    for (int64_t n0 = P / 2; n0 >= 1; n0 /= 2) {
        for (int64_t e = threadIdx.x; e < n0 * kp; e += blockDim.x) {
            const int64_t node = n0 + e / kp;
            const int c = (int)(e % kp);
            nm[node * kp + c] = nm[2 * node * kp + c] + nm[(2 * node + 1) * kp + c];
        }
        __syncthreads();
    }
}

template <class R>
__device__ __forceinline__ double frac_kernel(const double (&xs)[3], const double* y, double expo)
{
    R d[3];
    for (int m = 0; m < 3; ++m) d[m] = (R)(xs[m] - y[m]);
    const R r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
    if (sizeof(R) == sizeof(float))
        return (double)__builtin_amdgcn_exp2f((float)expo * __builtin_amdgcn_logf((float)r2));
    return pow((double)r2, expo);
}

template <class R, class UB, int KP>
__global__ __launch_bounds__(256) void k_bh_frac(BhArgs A, const UB* __restrict__ ub, int k,
                                                 const double* __restrict__ nm, double expo,
                                                 double* __restrict__ z, int64_t zstride)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool live = p < A.nF;                 // every lane walks with its wave
    const int32_t s = A.order[live ? p : 0];
    const double4 X = A.dx[s];
    const double xs[3] = {X.x, X.y, X.z};
    double slo[3], shi[3];
    for (int m = 0; m < 3; ++m) {
        slo[m] = A.flo[3 * s + m];
        shi[m] = A.fhi[3 * s + m];
    }
    const double sr2 = A.fr2[s];
    double us[KP], acc[KP];
    load_row<KP>(ub + (int64_t)s * KP, us);
#pragma unroll
    for (int c = 0; c < KP; ++c) acc[c] = 0.0;
    wave_walk(
        A.na, A.P, live, [&](int node) { return admissible(A, slo, shi, sr2, node); },
        [&](int node) {
            double m[KP];
            load_row<KP>(nm + (int64_t)node * KP, m);
            const double w = frac_kernel<R>(xs, A.nX + 3 * (int64_t)node, expo);
            const double a = A.na[node];
#pragma unroll
            for (int c = 0; c < KP; ++c) acc[c] += w * (a * us[c] - m[c]);
        },
        [&](int node) {
            const int64_t l = node - A.P;
            const int64_t p1 = min((l + 1) * (int64_t)A.leaf, A.nF);
            for (int64_t q = l * A.leaf; q < p1; ++q) {
                const int32_t t = A.order[q];
                if (t == s) continue;
                const double4 Y = A.dx[t];
                double ut[KP];
                load_row<KP>(ub + (int64_t)t * KP, ut);
                const double y[3] = {Y.x, Y.y, Y.z};
                const double w = frac_kernel<R>(xs, y, expo) * Y.w;
#pragma unroll
                for (int c = 0; c < KP; ++c) acc[c] += w * (us[c] - ut[c]);
            }
        });
    if (!live) return;
#pragma unroll
    for (int c = 0; c < KP; ++c)
        if (c < k) z[c * zstride + s] = acc[c];
}

template <class UB, int KP>
void moments_launch(const BhBuffers& b, int64_t nF, int leaf, int64_t P, const FaceData& fd, const UB* ub,
                    double* nm, hipStream_t s)
{
    hipLaunchKernelGGL((k_bh_moment_leaves<UB, KP>), dim3((unsigned)((P + 255) / 256)), dim3(256), 0, s, nF, leaf,
                       P, b.order, fd.dx, ub, nm);
    hipLaunchKernelGGL(k_bh_moment_levels, dim3(1), dim3(1024), 0, s, P, KP, nm);
}

template <class UB, int KP>
hipError_t bh_frac_launch(const BhBuffers& b, int64_t nF, int leaf, double theta, bool f64, const FaceData& fd,
                          const UB* ub, int k, double expo, double* nm, double* z, int64_t zstride, hipStream_t s)
{
    int64_t P = 0;
    (void)bh_node_count(nF, leaf, &P);
    moments_launch<UB, KP>(b, nF, leaf, P, fd, ub, nm, s);
    BhArgs A;
    A.nF = nF; A.P = P; A.leaf = leaf; A.theta2 = theta * theta; A.alpha = 0.0; A.beta = 0.0;
    A.order = b.order; A.dx = fd.dx; A.dn = fd.dn; A.flo = b.flo; A.fhi = b.fhi; A.fr2 = b.fr2;
    A.na = b.na; A.nX = b.nX; A.nlo = b.nlo; A.nhi = b.nhi; A.nr2 = b.nr2;
    A.gS = nullptr; A.eS = nullptr; A.accF = nullptr; A.accN = nullptr; A.counts = nullptr;
    // pair terms in the precision of the face averages (FP64 for TP_PREC_FP64, else FP32)
    (void)f64;
    const dim3 grid((unsigned)((nF + 255) / 256)), block(256);
    hipLaunchKernelGGL((k_bh_frac<UB, UB, KP>), grid, block, 0, s, A, ub, k, nm, expo, z, zstride);
    return hipGetLastError();
}

// ---------------------------------------------------------------- block cluster tree
//
// Hierarchical multiplication with the kernel matrix of the fractional operator (Sec.
// 5.1.4, 5.1.5, App. B) on the same tree: the block lists (admissible node pairs grouped by
// row node, inadmissible leaf pairs grouped by row leaf) are built on the host.  With
// x = [a, a ubar] per face and its node sums x~_J = [a_J, m_J] (the upward pass: the
// Barnes-Hut moments), y~_I = sum_{J admissible for I} k(X_I, X_J) x~_J (k_bct_far); face S
// then adds the y~ of its leaf and all its ancestors (the downward pass, summed along the
// face's path) and the exact terms of the leaves inadmissible for its own:
//   z(S) = ubar_S Y0(S) - Y(S) + sum_{T in near leaves, T != S} k(X_S, X_T) a_T (ubar_S - ubar_T).
// y~ rows are 4 + KP wide: [sum w a_J, 0, 0, 0, sum w m_J (KP)].

// Admissible blocks: one wave per row node I.  The lanes take the node's list in strides of
// 64 entries; the sums are then added across the wave in a fixed order (butterfly), so the
// result does not depend on timing.
template <class R, int KP>
__global__ __launch_bounds__(256) void k_bct_far(int64_t M, const int32_t* __restrict__ off,
                                                 const int32_t* __restrict__ col, const double* __restrict__ nX,
                                                 const double* __restrict__ na, const double* __restrict__ nm,
                                                 double expo, double* __restrict__ yt)
{
    const int64_t I = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int lane = threadIdx.x & 63;
    if (I >= M) return;                       // the whole wave
    double a0 = 0.0, acc[KP];
#pragma unroll
    for (int c = 0; c < KP; ++c) acc[c] = 0.0;
    const double xi[3] = {nX[3 * I], nX[3 * I + 1], nX[3 * I + 2]};
    const int32_t e1 = off[I + 1];
    for (int32_t e = off[I] + lane; e < e1; e += 64) {
        const int32_t J = col[e];
        double m[KP];
        load_row<KP>(nm + (int64_t)J * KP, m);
        const double w = frac_kernel<R>(xi, nX + 3 * J, expo);
        a0 += w * na[J];
#pragma unroll
        for (int c = 0; c < KP; ++c) acc[c] += w * m[c];
    }
    a0 = wave_sum(a0);
#pragma unroll
    for (int c = 0; c < KP; ++c) acc[c] = wave_sum(acc[c]);
    if (lane == 0) {
        double* y = yt + I * (KP + 4);
        y[0] = a0;
        y[1] = 0.0;
        y[2] = 0.0;
        y[3] = 0.0;
#pragma unroll
        for (int c = 0; c < KP; ++c) y[4 + c] = acc[c];
    }
}

// z(S) += ubar_S Y0 - Y over the leaf L's path to the root (downward pass)
template <int KP>
__device__ __forceinline__ void bct_down(const double* __restrict__ yt, int64_t P, int64_t L, const double (&us)[KP],
                                         double (&acc)[KP])
{
    double y0 = 0.0, yc[KP];
#pragma unroll
    for (int c = 0; c < KP; ++c) yc[c] = 0.0;
    for (int64_t node = P + L; node >= 1; node >>= 1) {
        const double* y = yt + node * (KP + 4);
        double v[KP];
        load_row<KP>(y + 4, v);
        y0 += y[0];
#pragma unroll
        for (int c = 0; c < KP; ++c) yc[c] += v[c];
    }
#pragma unroll
    for (int c = 0; c < KP; ++c) acc[c] += us[c] * y0 - yc[c];
}

// Inadmissible (exact) blocks for leaves of at most 8 faces: one wave per row leaf L, lane
// (i, j) = (lane / 8, lane % 8) takes the pair (face i of L, face j of J) for every leaf J of
// L's list, all lanes walking the same list (64 list entries are read at once and handed
// out lane by lane; the gathers of U leaves are issued before any of them is used); the 8
// lanes of face i are then added in a fixed order and lane (i, 0) adds the far field of L's
// path to the root.
template <class R, class UB, int KP>
__global__ __launch_bounds__(256) void k_bct_leaf8(int64_t nF, int leaf, int64_t P, const int32_t* __restrict__ order,
                                                   const double4* __restrict__ dx, const UB* __restrict__ ub, int k,
                                                   const int32_t* __restrict__ noff,
                                                   const int32_t* __restrict__ ncol, const double* __restrict__ yt,
                                                   double expo, double* __restrict__ z, int64_t zstride)
{
    constexpr int U = 4;
    const int64_t L = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int lane = threadIdx.x & 63;
    const int64_t nleaf = (nF + leaf - 1) / leaf;
    if (L >= nleaf) return;                   // the whole wave
    const int i = lane >> 3, j = lane & 7;
    const int64_t ps = L * leaf + i;
    const bool own = i < leaf && ps < nF;
    const bool lane_on = own && j < leaf;
    const int32_t s = own ? order[ps] : order[0];
    const double4 X = dx[s];
    const double xs[3] = {X.x, X.y, X.z};
    double us[KP], acc[KP];
    load_row<KP>(ub + (int64_t)s * KP, us);
#pragma unroll
    for (int c = 0; c < KP; ++c) acc[c] = 0.0;
    const int32_t e0 = noff[L], e1 = noff[L + 1];
    for (int32_t eb = e0; eb < e1; eb += 64) {
        const int32_t mine = eb + lane < e1 ? ncol[eb + lane] : 0;
        const int nb = min(64, e1 - eb);
        for (int q0 = 0; q0 < nb; q0 += U) {
            int32_t t[U];
#pragma unroll
            for (int q = 0; q < U; ++q) {
                const int32_t J = __shfl(mine, q0 + q, 64);
                const int64_t pt = (int64_t)J * leaf + j;
                t[q] = (lane_on && q0 + q < nb && pt < nF) ? order[pt] : -1;
            }
            double4 Y[U];
            double ut[U][KP];
#pragma unroll
            for (int q = 0; q < U; ++q) {
                const int32_t tq = t[q] >= 0 ? t[q] : s;
                Y[q] = dx[tq];
                load_row<KP>(ub + (int64_t)tq * KP, ut[q]);
            }
#pragma unroll
            for (int q = 0; q < U; ++q) {
                if (t[q] < 0 || t[q] == s) continue;
                const double y[3] = {Y[q].x, Y[q].y, Y[q].z};
                const double w = frac_kernel<R>(xs, y, expo) * Y[q].w;
#pragma unroll
                for (int c = 0; c < KP; ++c) acc[c] += w * (us[c] - ut[q][c]);
            }
        }
    }
#pragma unroll
    for (int c = 0; c < KP; ++c) {
        double v = acc[c];
        v += __shfl_xor(v, 4, 64);
        v += __shfl_xor(v, 2, 64);
        v += __shfl_xor(v, 1, 64);
        acc[c] = v;
    }
    if (!own || j != 0) return;
    bct_down<KP>(yt, P, L, us, acc);
#pragma unroll
    for (int c = 0; c < KP; ++c)
        if (c < k) z[c * zstride + s] = acc[c];
}

// The same for any leaf size: one thread per face, its leaf's list in order.
template <class R, class UB, int KP>
__global__ __launch_bounds__(256) void k_bct_faces(int64_t nF, int leaf, int64_t P, const int32_t* __restrict__ order,
                                                   const double4* __restrict__ dx, const UB* __restrict__ ub, int k,
                                                   const int32_t* __restrict__ noff,
                                                   const int32_t* __restrict__ ncol, const double* __restrict__ yt,
                                                   double expo, double* __restrict__ z, int64_t zstride)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= nF) return;
    const int32_t s = order[p];
    const double4 X = dx[s];
    const double xs[3] = {X.x, X.y, X.z};
    double us[KP], acc[KP];
    load_row<KP>(ub + (int64_t)s * KP, us);
#pragma unroll
    for (int c = 0; c < KP; ++c) acc[c] = 0.0;
    const int64_t L = p / leaf;
    for (int32_t e = noff[L]; e < noff[L + 1]; ++e) {
        const int64_t J = ncol[e];
        const int64_t q1 = min((J + 1) * (int64_t)leaf, nF);
        for (int64_t q = J * leaf; q < q1; ++q) {
            const int32_t t = order[q];
            if (t == s) continue;
            const double4 Y = dx[t];
            double ut[KP];
            load_row<KP>(ub + (int64_t)t * KP, ut);
            const double y[3] = {Y.x, Y.y, Y.z};
            const double w = frac_kernel<R>(xs, y, expo) * Y.w;
#pragma unroll
            for (int c = 0; c < KP; ++c) acc[c] += w * (us[c] - ut[c]);
        }
    }
    bct_down<KP>(yt, P, L, us, acc);
#pragma unroll
    for (int c = 0; c < KP; ++c)
        if (c < k) z[c * zstride + s] = acc[c];
}

template <class UB, int KP>
hipError_t bct_launch(const BhBuffers& b, const BctLists& bl, int64_t nF, int leaf, bool f64, const FaceData& fd,
                      const UB* ub, int k, double expo, double* nm, double* yt, double* z, int64_t zstride,
                      hipStream_t s)
{
    int64_t P = 0;
    const int64_t M = (int64_t)bh_node_count(nF, leaf, &P);
    moments_launch<UB, KP>(b, nF, leaf, P, fd, ub, nm, s);
    // one wave (64 lanes) per node for the admissible blocks, per leaf for the exact ones
    const int64_t nleaf = (nF + leaf - 1) / leaf;
    const dim3 gm((unsigned)((M * 64 + 255) / 256)), gl((unsigned)((nleaf * 64 + 255) / 256)),
        gf((unsigned)((nF + 255) / 256)), blk(256);
    // pair terms in the precision of the face averages (FP64 for TP_PREC_FP64, else FP32)
    (void)f64;
    hipLaunchKernelGGL((k_bct_far<UB, KP>), gm, blk, 0, s, M, bl.far_off, bl.far_col, b.nX, b.na, nm, expo, yt);
    if (leaf <= 8)
        hipLaunchKernelGGL((k_bct_leaf8<UB, UB, KP>), gl, blk, 0, s, nF, leaf, P, b.order, fd.dx, ub, k, bl.near_off,
                           bl.near_col, yt, expo, z, zstride);
    else
        hipLaunchKernelGGL((k_bct_faces<UB, UB, KP>), gf, blk, 0, s, nF, leaf, P, b.order, fd.dx, ub, k, bl.near_off,
                           bl.near_col, yt, expo, z, zstride);
    return hipGetLastError();
}

// ---------------------------------------------------------------- block cluster tree lists
//
// The blocks of the fractional operator's kernel matrix, built on the device by a
// breadth-first split of (root, root): a pair of nodes of one depth is an admissible block
// when separated, an exact block when it is a pair of leaves, else its four pairs of
// children go to the next level.  Appends use atomic counters, so the order in which a
// level's blocks land is arbitrary; the lists are then sorted by (row, column), which fixes
// them.  The separation test repeats the reading's arithmetic in FP64 without fused
// multiply-adds, as for the Barnes-Hut admissibility.
// Node records for the split: lo (3), hi (3), r^2, a_I -- one 64-byte line per node, since
// the pairs of a level reach their nodes in no cache-friendly order.
__global__ void k_bct_nodes(int64_t M, const double* __restrict__ na, const double* __restrict__ nlo,
                            const double* __restrict__ nhi, const double* __restrict__ nr2, double* __restrict__ rec)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= M) return;
    double* r = rec + 8 * i;
    for (int m = 0; m < 3; ++m) {
        r[m] = nlo[3 * i + m];
        r[3 + m] = nhi[3 * i + m];
    }
    r[6] = nr2[i];
    r[7] = na[i];
}

__device__ __forceinline__ bool bct_separated(const double (&a)[8], const double (&b)[8], double chi2)
{
    double d2 = 0.0;
    for (int m = 0; m < 3; ++m) {
        const double g1 = b[m] - a[3 + m];
        const double g2 = a[m] - b[3 + m];
        double g = g1 > g2 ? g1 : g2;
        g = g < 0.0 ? 0.0 : g;
        d2 = d2 + g * g;
    }
    const double r2 = a[6] > b[6] ? a[6] : b[6];
    return r2 < chi2 * d2;
}

// One level of the split: each thread takes kExpPer pairs; the block counts its appends
// per list (wave prefix sums, then across the block's waves) and reserves them with one
// atomic addition per list, so same-address atomics stay few.
// cnt[0], cnt[1]: admissible and exact blocks so far (appended at these positions);
// cnt[2]: pairs of the next level.
constexpr int kExpThreads = 1024, kExpPer = 4;

__global__ __launch_bounds__(kExpThreads) void k_bct_expand(const uint64_t* __restrict__ cur, int64_t n,
                                                            const double4* __restrict__ rec, int64_t P, double chi2,
                                                            uint64_t* __restrict__ far, uint64_t* __restrict__ near,
                                                            uint64_t* __restrict__ next,
                                                            unsigned long long* __restrict__ cnt)
{
    __shared__ unsigned long long wsum[3][kExpThreads / 64];
    __shared__ unsigned long long base[3];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int64_t e0 = (int64_t)blockIdx.x * kExpThreads * kExpPer + tid;
    uint64_t key[kExpPer];
    int what[kExpPer];                          // 1 admissible, 2 exact, 3 split, 0 nothing
    unsigned long long c[3] = {0ull, 0ull, 0ull};
#pragma unroll
    for (int q = 0; q < kExpPer; ++q) {
        const int64_t e = e0 + (int64_t)q * kExpThreads;
        key[q] = 0;
        what[q] = 0;
        if (e < n) {
            key[q] = cur[e];
            const int64_t I = (int64_t)(key[q] >> 32), J = (int64_t)(key[q] & 0xffffffffull);
            const double4 a0 = rec[2 * I], a1 = rec[2 * I + 1], b0 = rec[2 * J], b1 = rec[2 * J + 1];
            const double av[8] = {a0.x, a0.y, a0.z, a0.w, a1.x, a1.y, a1.z, a1.w};
            const double bv[8] = {b0.x, b0.y, b0.z, b0.w, b1.x, b1.y, b1.z, b1.w};
            if (av[7] > 0.0 && bv[7] > 0.0)
                what[q] = bct_separated(av, bv, chi2) ? 1 : (I >= P ? 2 : 3);   // pairs stay on one depth
        }
        if (what[q]) c[what[q] - 1] += what[q] == 3 ? 4ull : 1ull;
    }
    unsigned long long incl[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        unsigned long long v = c[k];
        for (int o = 1; o < 64; o <<= 1) {
            const unsigned long long t = __shfl_up(v, o, 64);
            if (lane >= o) v += t;
        }
        incl[k] = v;
        if (lane == 63) wsum[k][wid] = v;
    }
    __syncthreads();
    if (tid < 3) {
        unsigned long long tot = 0ull;
        for (int w = 0; w < kExpThreads / 64; ++w) {
            const unsigned long long v = wsum[tid][w];
            wsum[tid][w] = tot;
            tot += v;
        }
        base[tid] = tot ? atomicAdd(&cnt[tid], tot) : 0ull;
    }
    __syncthreads();
    unsigned long long off[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) off[k] = base[k] + wsum[k][wid] + incl[k] - c[k];
#pragma unroll
    for (int q = 0; q < kExpPer; ++q) {
        const int64_t I = (int64_t)(key[q] >> 32), J = (int64_t)(key[q] & 0xffffffffull);
        if (what[q] == 1) {
            far[off[0]++] = key[q];
        } else if (what[q] == 2) {
            near[off[1]++] = ((uint64_t)(I - P) << 32) | (uint64_t)(J - P);
        } else if (what[q] == 3) {
            for (int a = 0; a < 2; ++a)
                for (int b = 0; b < 2; ++b)
                    next[off[2] + 2 * a + b] = ((uint64_t)(2 * I + a) << 32) | (uint64_t)(2 * J + b);
            off[2] += 4;
        }
    }
}

// CSR of sorted (row << 32 | column) keys: off[r] = first key of row r (r = 0 .. rows),
// col[e] = column of key e.
__global__ void k_bct_csr(const uint64_t* __restrict__ keys, int64_t n, int64_t rows, int32_t* __restrict__ off,
                          int32_t* __restrict__ col)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t <= rows) {
        const uint64_t target = (uint64_t)t << 32;
        int64_t lo = 0, hi = n;
        while (lo < hi) {
            const int64_t mid = (lo + hi) >> 1;
            if (keys[mid] < target) lo = mid + 1;
            else hi = mid;
        }
        off[t] = (int32_t)lo;
    }
    if (t < n) col[t] = (int32_t)(keys[t] & 0xffffffffull);
}

}  // namespace

size_t bh_node_count(int64_t nF, int leaf, int64_t* P_out)
{
    const int64_t nleaf = (nF + leaf - 1) / leaf;
    int64_t P = 1;
    while (P < nleaf) P *= 2;
    if (P_out) *P_out = P;
    return (size_t)(2 * P);
}

size_t bh_sort_temp_bytes(int64_t nF)
{
    size_t bytes = 0;
    (void)hipcub::DeviceRadixSort::SortPairs(nullptr, bytes, (const uint64_t*)nullptr, (uint64_t*)nullptr,
                                             (const int32_t*)nullptr, (int32_t*)nullptr, (int)nF, 0, 62);
    return bytes;
}

hipError_t launch_morton_order(const BhBuffers& b, const FaceData& fd, int64_t nF, const int32_t* orig,
                               hipStream_t s)
{
    const unsigned g = (unsigned)((nF + 255) / 256);
    hipLaunchKernelGGL(k_bh_bbox, dim3(1), dim3(1024), 0, s, fd.dx, nF, b.box);
    // values in b.pos, sorted values into b.order
    hipLaunchKernelGGL(k_bh_keys, dim3(g), dim3(256), 0, s, fd.dx, nF, b.box, orig, b.keys_in, b.pos);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    size_t tb = b.sort_bytes;
    return hipcub::DeviceRadixSort::SortPairs(b.sort_tmp, tb, b.keys_in, b.keys_out, b.pos, b.order, (int)nF, 0, 62, s);
}

hipError_t launch_bh_build(const BhBuffers& b, const double* V, const int32_t* F, const int32_t* orig, int64_t nF,
                           int leaf, const FaceData& fd, hipStream_t s)
{
    int64_t P = 0;
    (void)bh_node_count(nF, leaf, &P);
    const unsigned g = (unsigned)((nF + 255) / 256);
    hipLaunchKernelGGL(k_bh_faceprep, dim3(g), dim3(256), 0, s, V, F, nF, fd.dx, b.flo, b.fhi, b.fr2);
    hipError_t e = launch_morton_order(b, fd, nF, orig, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_bh_pos, dim3(g), dim3(256), 0, s, b.order, nF, b.pos);
    hipLaunchKernelGGL(k_bh_leaves, dim3((unsigned)((P + 255) / 256)), dim3(256), 0, s, nF, leaf, P, b.order,
                       fd.dx, b.flo, b.fhi, b.na, b.nsx, b.nlo, b.nhi);
    hipLaunchKernelGGL(k_bh_levels, dim3(1), dim3(1024), 0, s, P, b.na, b.nsx, b.nlo, b.nhi, b.nX, b.nr2);
    return hipGetLastError();
}

hipError_t launch_bh_eval(const BhBuffers& b, int64_t nF, int leaf, double theta, int precision, double alpha,
                          double beta, const FaceData& fd, bool grad, double* gface, int64_t gstride,
                          hipStream_t s)
{
    int64_t P = 0;
    const int64_t M = (int64_t)bh_node_count(nF, leaf, &P);
    hipError_t e = hipMemsetAsync(b.counts, 0, 2 * sizeof(unsigned long long), s);
    if (e != hipSuccess) return e;
    if (grad) {
        if ((e = hipMemsetAsync(b.accF, 0, sizeof(double) * 4 * nF, s)) != hipSuccess) return e;
        if ((e = hipMemsetAsync(b.accN, 0, sizeof(double) * 4 * M, s)) != hipSuccess) return e;
    }
    BhArgs A;
    A.nF = nF; A.P = P; A.leaf = leaf; A.theta2 = theta * theta; A.alpha = alpha; A.beta = beta;
    A.order = b.order; A.dx = fd.dx; A.dn = fd.dn; A.flo = b.flo; A.fhi = b.fhi; A.fr2 = b.fr2;
    A.na = b.na; A.nX = b.nX; A.nlo = b.nlo; A.nhi = b.nhi; A.nr2 = b.nr2;
    A.gS = b.gS; A.eS = b.eS; A.accF = b.accF; A.accN = b.accN; A.counts = b.counts;
    const dim3 grid((unsigned)((nF + 255) / 256)), block(256);
    const bool gen = !(alpha == 6.0 && beta == 12.0);
    const bool f64 = precision == TP_PREC_FP64;
#define TP_BH_LAUNCH(R, G, D) hipLaunchKernelGGL((k_bh_traverse<R, G, D>), grid, block, 0, s, A)
    if (grad) {
        if (f64) { if (gen) TP_BH_LAUNCH(double, true, true); else TP_BH_LAUNCH(double, false, true); }
        else { if (gen) TP_BH_LAUNCH(float, true, true); else TP_BH_LAUNCH(float, false, true); }
    } else {
        if (f64) { if (gen) TP_BH_LAUNCH(double, true, false); else TP_BH_LAUNCH(double, false, false); }
        else { if (gen) TP_BH_LAUNCH(float, true, false); else TP_BH_LAUNCH(float, false, false); }
    }
#undef TP_BH_LAUNCH
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (grad)
        hipLaunchKernelGGL(k_bh_assemble, grid, block, 0, s, nF, leaf, P, b.pos, fd.dx, b.na, b.nX, b.gS, b.accF,
                           b.accN, gface, gstride);
    return hipGetLastError();
}

hipError_t launch_bh_frac(const BhBuffers& b, int64_t nF, int leaf, double theta, int precision, double sigma,
                          const FaceData& fd, const void* ub, int kp, int k, double* nm, double* z, int64_t zstride,
                          hipStream_t s)
{
    if (k < 1 || k > kMaxGroupCols || kp != (k + 3) / 4 * 4) return hipErrorInvalidValue;
    const double expo = -(sigma + 1.0);
    const bool f64 = precision == TP_PREC_FP64;
#define TP_BHF(T, KP) bh_frac_launch<T, KP>(b, nF, leaf, theta, f64, fd, static_cast<const T*>(ub), k, expo, nm, z, zstride, s)
    if (f64) return kp == 4 ? TP_BHF(double, 4) : kp == 8 ? TP_BHF(double, 8) : TP_BHF(double, 12);
    return kp == 4 ? TP_BHF(float, 4) : kp == 8 ? TP_BHF(float, 8) : TP_BHF(float, 12);
#undef TP_BHF
}

hipError_t launch_bct_frac(const BhBuffers& b, const BctLists& bl, int64_t nF, int leaf, int precision,
                           double sigma, const FaceData& fd, const void* ub, int kp, int k, double* nm, double* yt,
                           double* z, int64_t zstride, hipStream_t s)
{
    if (k < 1 || k > kMaxGroupCols || kp != (k + 3) / 4 * 4) return hipErrorInvalidValue;
    const double expo = -(sigma + 1.0);
    const bool f64 = precision == TP_PREC_FP64;
#define TP_BCT(T, KP) bct_launch<T, KP>(b, bl, nF, leaf, f64, fd, static_cast<const T*>(ub), k, expo, nm, yt, z, zstride, s)
    if (f64) return kp == 4 ? TP_BCT(double, 4) : kp == 8 ? TP_BCT(double, 8) : TP_BCT(double, 12);
    return kp == 4 ? TP_BCT(float, 4) : kp == 8 ? TP_BCT(float, 8) : TP_BCT(float, 12);
#undef TP_BCT
}

size_t bct_sort_temp_bytes(int64_t n)
{
    size_t bytes = 0;
    (void)hipcub::DeviceRadixSort::SortKeys(nullptr, bytes, (const uint64_t*)nullptr, (uint64_t*)nullptr,
                                            (int)std::max<int64_t>(n, 1), 0, 64);
    return bytes;
}

hipError_t launch_bct_nodes(const BhBuffers& b, int64_t M, double* rec, hipStream_t s)
{
    hipLaunchKernelGGL(k_bct_nodes, dim3((unsigned)((M + 255) / 256)), dim3(256), 0, s, M, b.na, b.nlo, b.nhi, b.nr2,
                       rec);
    return hipGetLastError();
}

hipError_t launch_bct_expand(const double* rec, int64_t P, double chi, const uint64_t* cur, int64_t n, uint64_t* far,
                             uint64_t* near, uint64_t* next, unsigned long long* cnt, hipStream_t s)
{
    if (n < 1) return hipSuccess;
    const int64_t per_block = (int64_t)kExpThreads * kExpPer;
    hipLaunchKernelGGL(k_bct_expand, dim3((unsigned)((n + per_block - 1) / per_block)), dim3(kExpThreads), 0, s, cur,
                       n, reinterpret_cast<const double4*>(rec), P, chi * chi, far, near, next, cnt);
    return hipGetLastError();
}

hipError_t launch_bct_sort_csr(const uint64_t* keys, uint64_t* sorted, int64_t n, void* tmp, size_t tmp_bytes,
                               int64_t rows, int32_t* off, int32_t* col, hipStream_t s)
{
    if (n > (int64_t)INT32_MAX) return hipErrorInvalidValue;
    if (n > 0) {
        size_t tb = tmp_bytes;
        hipError_t e = hipcub::DeviceRadixSort::SortKeys(tmp, tb, keys, sorted, (int)n, 0, 64, s);
        if (e != hipSuccess) return e;
    }
    const int64_t m = std::max(rows + 1, n);
    hipLaunchKernelGGL(k_bct_csr, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s, sorted, n, rows, off, col);
    return hipGetLastError();
}

}  // namespace tp

