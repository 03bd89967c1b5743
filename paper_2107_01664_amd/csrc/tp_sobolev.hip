// The inner-product operator A = B + B0 (Sec. 2.4; discrete terms in Sec. 3.2.1, eqs.
// DiscreteHighOrderTerm and DiscreteLowOrderTerm), applied in the factored form of
// Sec. 5.1.2 and 5.1.3:
//
//   A u = 2 (diag(a) D)^T [diag(diag(a)^-1 H a) - H] (diag(a) D) u
//       + 2 U^T [diag(diag(a)^-1 H0 a) - H0] U u,
//
// H_ST = |X_S - X_T|^-2s (sigma = s - 1), H0_ST = H_ST (K2(S,T) + K2(T,S)) / 2 with
// K2(S,T) = (N_S . d)^2 / |d|^4 (the tangent-point kernel with exponents 2 and 4), D u(S)
// the gradient of the piecewise linear u on face S, U the face average times the area.
// Row S of a bracket applied to diag(a) v is sum_{T != S} H_ST a_T (v(S) - v(T)).
//
// Three passes per group of kc <= kSobCols columns:
//   k_sob_face    per face and column: D u (3 values) and ubar, from V and F in FP64, stored
//                 as one FP32 (or FP64) 4-vector per column, [cap][kc];
//   k_sob32/64    the pair sums with the tiling of the other all-pairs kernels: an i-tile of
//                 kBlock * NI faces in registers, j-tiles of kTileJ faces through LDS (every
//                 lane reads the same face T), an (i-tiles) x (j-splits) grid whose partial
//                 sums per split are added in order by launch_reduce_splits.  Per pair: d
//                 (hi/lo), r2, w = r2^-s a_T by log2/exp2, q_S = N_S . d, q_T = N_T . d,
//                 w0 = w (q_S^2 + q_T^2) / r2^2; zB += w (D u(S) - D u(T)), z0 += w0 (ubar(S) - ubar(T));
//   k_sob_gather  (A u)_i = sum over the faces S around i of 2 a_S (<D phi_i(S), zB(S)> + z0(S) / 6)
//                 (the 1/2 of the symmetrized K2 and phibar = 1/3 give the 1/6), with
//                 D phi_i(S) = c_S x (f_k - f_j) / |c_S|^2 in FP64 for the corners i, j, k of
//                 S in cyclic order, c_S = (f_j - f_i) x (f_k - f_i).
//
// The diagonal S = T contributes nothing: d = 0 there, so both differences and q vanish;
// r2 is set to 1 on it to keep the powers finite.
#include "tp_sobolev.h"
#include "tp_sym.h"
#include "tp_tiles.h"

#include <algorithm>
#include <mutex>
#include <unordered_map>

namespace tp {

namespace {

inline unsigned nblk(int64_t n, int b = 256) { return (unsigned)((n + b - 1) / b); }

constexpr int kNiSob32 = 2;

struct SobArgs {
    const void* fx;     // float4 (Xhi, a) or double4 (X, a)
    const void* fl;     // float4 (Xlo, 0)
    const void* fn;     // float4 or double4 (N, 0)
    const void* fu;     // [cap][KC] 4-vectors (D u, ubar)
    double* part;       // [n_split][4 KC][irows]
    const float4* tbox; // per-tile boxes of the FP32 barycenters (far-tile test)
    int64_t irows;
    int n_itiles, tiles_per_split, ntiles_j;
};

__device__ __forceinline__ bool hits_diag(int64_t j0, int64_t ibase, int ispan)
{
    return j0 < ibase + ispan && j0 + kTileJ > ibase;
}

// ------------------------------------------------------------------ per-face columns

template <class R, class R4>
__global__ void k_sob_face(const double* __restrict__ V, const int32_t* __restrict__ F, int64_t nF,
                           int64_t cap, const double* __restrict__ u, int ldu, int kc, R4* __restrict__ fu)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= cap) return;
    if (t >= nF) {
        for (int c = 0; c < kc; ++c) fu[t * kc + c] = R4{0, 0, 0, 0};
        return;
    }
    int32_t id[3];
    double p[3][3];
    for (int m = 0; m < 3; ++m) {
        id[m] = F[3 * t + m];
        for (int x = 0; x < 3; ++x) p[m][x] = V[3 * (int64_t)id[m] + x];
    }
    const double e1[3] = {p[1][0] - p[0][0], p[1][1] - p[0][1], p[1][2] - p[0][2]};
    const double e2[3] = {p[2][0] - p[0][0], p[2][1] - p[0][1], p[2][2] - p[0][2]};
    const double cr[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2],
                          e1[0] * e2[1] - e1[1] * e2[0]};
    const double ic2 = 1.0 / (cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2]);
    double g[3][3];   // D phi of each corner
    for (int m = 0; m < 3; ++m) {
        const double* pj = p[(m + 1) % 3];
        const double* pk = p[(m + 2) % 3];
        const double e[3] = {pk[0] - pj[0], pk[1] - pj[1], pk[2] - pj[2]};
        g[m][0] = (cr[1] * e[2] - cr[2] * e[1]) * ic2;
        g[m][1] = (cr[2] * e[0] - cr[0] * e[2]) * ic2;
        g[m][2] = (cr[0] * e[1] - cr[1] * e[0]) * ic2;
    }
    for (int c = 0; c < kc; ++c) {
        const double u0 = u[(int64_t)id[0] * ldu + c], u1 = u[(int64_t)id[1] * ldu + c],
                     u2 = u[(int64_t)id[2] * ldu + c];
        R4 o;
        o.x = (R)(u0 * g[0][0] + u1 * g[1][0] + u2 * g[2][0]);
        o.y = (R)(u0 * g[0][1] + u1 * g[1][1] + u2 * g[2][1]);
        o.z = (R)(u0 * g[0][2] + u1 * g[1][2] + u2 * g[2][2]);
        o.w = (R)((u0 + u1 + u2) / 3.0);
        fu[t * kc + c] = o;
    }
}

// ------------------------------------------------------------------ FP32 pair sums

template <bool DIAG, int NI, int KC, bool HILO, bool ROWSUM>
__device__ __forceinline__ void sob_tile32(const float4* s_x, const float4* s_l, const float4* s_n,
                                           const float4* s_u, int64_t j0, const float3 (&Sh)[NI],
                                           const float3 (&Sl)[NI], const float3 (&Sn)[NI],
                                           const float4 (&Su)[NI][KC], const int64_t (&Si)[NI], float ms,
                                           float (&c)[NI][4 * KC])
{
    for (int jj = 0; jj < kTileJ; ++jj) {
        const float4 tx = s_x[jj];
        const float4 tn = s_n[jj];
        const float4 tl = HILO ? s_l[jj] : make_float4(0.f, 0.f, 0.f, 0.f);
        float4 tu[KC];
#pragma unroll
        for (int cc = 0; cc < KC; ++cc) tu[cc] = s_u[jj * KC + cc];
#pragma unroll
        for (int r = 0; r < NI; ++r) {
            float dx, dy, dz;
            if (HILO) {
                dx = (Sh[r].x - tx.x) + (Sl[r].x - tl.x);
                dy = (Sh[r].y - tx.y) + (Sl[r].y - tl.y);
                dz = (Sh[r].z - tx.z) + (Sl[r].z - tl.z);
            } else {
                dx = Sh[r].x - tx.x;
                dy = Sh[r].y - tx.y;
                dz = Sh[r].z - tx.z;
            }
            float r2 = dx * dx + dy * dy + dz * dz;
            if (DIAG) r2 = (Si[r] == j0 + jj) ? 1.0f : r2;
            const float w = __builtin_amdgcn_exp2f(ms * __builtin_amdgcn_logf(r2)) * tx.w;
            const float qs = Sn[r].x * dx + Sn[r].y * dy + Sn[r].z * dz;
            const float qt = tn.x * dx + tn.y * dy + tn.z * dz;
            const float inv = __builtin_amdgcn_rcpf(r2);
            const float w0 = w * ((qs * qs + qt * qt) * (inv * inv));
            if (ROWSUM) {   // the row sums of both kernel matrices (weights a_T included)
                c[r][0] += DIAG && Si[r] == j0 + jj ? 0.f : w;
                c[r][3] += w0;
                continue;
            }
#pragma unroll
            for (int cc = 0; cc < KC; ++cc) {
                c[r][4 * cc + 0] += w * (Su[r][cc].x - tu[cc].x);
                c[r][4 * cc + 1] += w * (Su[r][cc].y - tu[cc].y);
                c[r][4 * cc + 2] += w * (Su[r][cc].z - tu[cc].z);
                c[r][4 * cc + 3] += w0 * (Su[r][cc].w - tu[cc].w);
            }
        }
    }
}

template <int NI, int KC, bool HILO, bool ROWSUM = false>
__global__ __launch_bounds__(kBlock) void k_sob32(SobArgs A, float ms)
{
    const int bi = (int)blockIdx.x % A.n_itiles;
    const int bs = (int)blockIdx.x / A.n_itiles;
    const float4* __restrict__ fx = static_cast<const float4*>(A.fx);
    const float4* __restrict__ fl = static_cast<const float4*>(A.fl);
    const float4* __restrict__ fn = static_cast<const float4*>(A.fn);
    const float4* __restrict__ fu = static_cast<const float4*>(A.fu);
    __shared__ float4 s_x[kTileJ], s_l[HILO ? kTileJ : 1], s_n[kTileJ], s_u[kTileJ * KC];
    const int64_t ibase = (int64_t)bi * (kBlock * NI);
    const int jt0 = bs * A.tiles_per_split;
    const int jt1 = min(jt0 + A.tiles_per_split, A.ntiles_j);
    float3 Sh[NI], Sl[NI], Sn[NI];
    float4 Su[NI][KC];
    int64_t Si[NI];
    double acc[NI][4 * KC];
#pragma unroll
    for (int r = 0; r < NI; ++r) {
        Si[r] = ibase + r * kBlock + threadIdx.x;
        const float4 x = fx[Si[r]], n = fn[Si[r]];
        Sh[r] = make_float3(x.x, x.y, x.z);
        Sn[r] = make_float3(n.x, n.y, n.z);
        if (HILO) {
            const float4 l = fl[Si[r]];
            Sl[r] = make_float3(l.x, l.y, l.z);
        } else {
            Sl[r] = make_float3(0.f, 0.f, 0.f);
        }
#pragma unroll
        for (int cc = 0; cc < KC; ++cc) Su[r][cc] = ROWSUM ? make_float4(0.f, 0.f, 0.f, 0.f) : fu[Si[r] * KC + cc];
#pragma unroll
        for (int q = 0; q < 4 * KC; ++q) acc[r][q] = 0.0;
    }
    float4 ilo, ihi;
    if (HILO) irange_box(A.tbox, ibase, kBlock * NI, ilo, ihi);
    for (int jt = jt0; jt < jt1; ++jt) {
        const int64_t j0 = (int64_t)jt * kTileJ;
        __syncthreads();
        for (int e = threadIdx.x; e < kTileJ; e += kBlock) {
            s_x[e] = fx[j0 + e];
            s_n[e] = fn[j0 + e];
            if (HILO) s_l[e] = fl[j0 + e];
        }
        if (!ROWSUM)
            for (int e = threadIdx.x; e < kTileJ * KC; e += kBlock) s_u[e] = fu[j0 * KC + e];
        __syncthreads();
        float c[NI][4 * KC];
#pragma unroll
        for (int r = 0; r < NI; ++r)
#pragma unroll
            for (int q = 0; q < 4 * KC; ++q) c[r][q] = 0.f;
        if (hits_diag(j0, ibase, kBlock * NI))
            sob_tile32<true, NI, KC, HILO, ROWSUM>(s_x, s_l, s_n, s_u, j0, Sh, Sl, Sn, Su, Si, ms, c);
        else if (HILO && tile_is_far(ilo, ihi, A.tbox, jt))   // far tiles: the high parts suffice
            sob_tile32<false, NI, KC, false, ROWSUM>(s_x, s_l, s_n, s_u, j0, Sh, Sl, Sn, Su, Si, ms, c);
        else
            sob_tile32<false, NI, KC, HILO, ROWSUM>(s_x, s_l, s_n, s_u, j0, Sh, Sl, Sn, Su, Si, ms, c);
#pragma unroll
        for (int r = 0; r < NI; ++r)
#pragma unroll
            for (int q = 0; q < 4 * KC; ++q) acc[r][q] += (double)c[r][q];
    }
#pragma unroll
    for (int r = 0; r < NI; ++r)
#pragma unroll
        for (int q = 0; q < 4 * KC; ++q) A.part[((int64_t)bs * 4 * KC + q) * A.irows + Si[r]] = acc[r][q];
}

// ------------------------------------------------------------------ symmetric FP32 pair sums
//
// Both kernel matrices are symmetric up to the areas: H_ST a_T and H0_ST a_T use
// g = r2^-s and g0 = g (q_S^2 + q_T^2) / r2^2, which row T forms from the same bits (d
// changes sign exactly in FP32, and only squares of it and of the q enter).  So each
// unordered pair is evaluated once for both rows, as in the symmetric E + dE kernel: a wave
// holds the kSymNI faces S of block a in each lane and passes the faces T of block b along
// the wave with their columns and their own sums (row T's sums collect g a_S (v(S) - v(T)),
// the negation of its terms, and are negated on the store).  Partial sums per face and
// slice (4 kc of them) go to the banded FP32 buffers of the other symmetric kernels and are
// reduced in slice order by launch_reduce_sym_band.

struct SobSymArgs {
    const float4* fx = nullptr;
    const float4* fl = nullptr;
    const float4* fn = nullptr;
    const float4* fu = nullptr;   // [cap][KC]
    const float4* tbox = nullptr;
    float* part = nullptr;        // row T's sums: [K][4 KC][ldp]
    float* partS = nullptr;       // row S's sums: [nB][4 KC][ldS]
    int64_t ldp = 0, ldS = 0;
    int nB = 0, a0 = 0, a1 = 0;
};

template <int KC, bool LO, bool DIAG>
__device__ __forceinline__ void sob_sym_unit(const SobSymArgs& A, int a, int b, int lane, float ms,
                                             const float3 (&Sh)[kSymNI], const float3 (&Sl)[kSymNI],
                                             const float3 (&Sn)[kSymNI], const float (&aS)[kSymNI],
                                             const float4 (&Su)[kSymNI][KC], float (&sacc)[kSymNI][4 * KC])
{
    const WaveRot rot(lane);
    for (int q = 0; q < kSymFaces / 64; ++q) {
        const int64_t T = (int64_t)b * kSymFaces + q * 64 + lane;
        float4 th = A.fx[T];
        float3 tl = make_float3(0.f, 0.f, 0.f);
        if (LO) {
            const float4 l = A.fl[T];
            tl = make_float3(l.x, l.y, l.z);
        }
        const float4 n4 = A.fn[T];
        float3 tn = make_float3(n4.x, n4.y, n4.z);
        float4 tu[KC];
        float tacc[4 * KC];
#pragma unroll
        for (int c = 0; c < KC; ++c) tu[c] = A.fu[T * KC + c];
#pragma unroll
        for (int m = 0; m < 4 * KC; ++m) tacc[m] = 0.f;
        int ti = (int)T;
#pragma unroll 1
        for (int step = 0; step < 64; ++step) {
#pragma unroll
            for (int r = 0; r < kSymNI; ++r) {
                float dx, dy, dz;
                if (LO) {
                    dx = (Sh[r].x - th.x) + (Sl[r].x - tl.x);
                    dy = (Sh[r].y - th.y) + (Sl[r].y - tl.y);
                    dz = (Sh[r].z - th.z) + (Sl[r].z - tl.z);
                } else {
                    dx = Sh[r].x - th.x;
                    dy = Sh[r].y - th.y;
                    dz = Sh[r].z - th.z;
                }
                float r2 = dx * dx + dy * dy + dz * dz;
                if (DIAG) r2 = ((int)((int64_t)a * kSymFaces + r * 64 + lane) == ti) ? 1.0f : r2;
                const float g = __builtin_amdgcn_exp2f(ms * __builtin_amdgcn_logf(r2));
                const float qs = Sn[r].x * dx + Sn[r].y * dy + Sn[r].z * dz;
                const float qt = tn.x * dx + tn.y * dy + tn.z * dz;
                const float inv = __builtin_amdgcn_rcpf(r2);
                const float g0 = g * ((qs * qs + qt * qt) * (inv * inv));
                const float wT = g * th.w, w0T = g0 * th.w;
                const float wS = g * aS[r], w0S = g0 * aS[r];
#pragma unroll
                for (int c = 0; c < KC; ++c) {
                    const float ex = Su[r][c].x - tu[c].x, ey = Su[r][c].y - tu[c].y;
                    const float ez = Su[r][c].z - tu[c].z, ew = Su[r][c].w - tu[c].w;
                    sacc[r][4 * c + 0] += wT * ex;
                    sacc[r][4 * c + 1] += wT * ey;
                    sacc[r][4 * c + 2] += wT * ez;
                    sacc[r][4 * c + 3] += w0T * ew;
                    if (!DIAG) {   // minus row T's terms (negated on the store)
                        tacc[4 * c + 0] += wS * ex;
                        tacc[4 * c + 1] += wS * ey;
                        tacc[4 * c + 2] += wS * ez;
                        tacc[4 * c + 3] += w0S * ew;
                    }
                }
            }
            th.x = rot(th.x);
            th.y = rot(th.y);
            th.z = rot(th.z);
            th.w = rot(th.w);
            if (LO) {
                tl.x = rot(tl.x);
                tl.y = rot(tl.y);
                tl.z = rot(tl.z);
            }
            tn.x = rot(tn.x);
            tn.y = rot(tn.y);
            tn.z = rot(tn.z);
#pragma unroll
            for (int c = 0; c < KC; ++c) {
                tu[c].x = rot(tu[c].x);
                tu[c].y = rot(tu[c].y);
                tu[c].z = rot(tu[c].z);
                tu[c].w = rot(tu[c].w);
            }
            if (!DIAG) {
#pragma unroll
                for (int m = 0; m < 4 * KC; ++m) tacc[m] = rot(tacc[m]);
            }
            if (DIAG) ti = rot(ti);
        }
        // 64 rotations later every face T is back in its own lane
        if (!DIAG) {
#pragma unroll
            for (int m = 0; m < 4 * KC; ++m) A.part[((int64_t)(a - A.a0) * 4 * KC + m) * A.ldp + T] = -tacc[m];
        }
    }
}

template <int KC, bool HILO>
__global__ __launch_bounds__(kBlock) void k_sob32_sym(SobSymArgs A, float ms)
{
    const int lane = (int)threadIdx.x & 63;
    const int64_t unit = (int64_t)blockIdx.x * (kBlock / 64) + ((int)threadIdx.x >> 6);
    int a, b;
    if (!sym_unit_blocks(unit, A.nB, A.a0, A.a1, a, b)) return;   // the whole wave leaves
    float3 Sh[kSymNI], Sl[kSymNI], Sn[kSymNI];
    float aS[kSymNI], sacc[kSymNI][4 * KC];
    float4 Su[kSymNI][KC];
#pragma unroll
    for (int r = 0; r < kSymNI; ++r) {
        const int64_t S = (int64_t)a * kSymFaces + r * 64 + lane;
        const float4 x = A.fx[S], n = A.fn[S];
        Sh[r] = make_float3(x.x, x.y, x.z);
        Sn[r] = make_float3(n.x, n.y, n.z);
        aS[r] = x.w;
        if (HILO) {
            const float4 l = A.fl[S];
            Sl[r] = make_float3(l.x, l.y, l.z);
        } else {
            Sl[r] = make_float3(0.f, 0.f, 0.f);
        }
#pragma unroll
        for (int c = 0; c < KC; ++c) Su[r][c] = A.fu[S * KC + c];
#pragma unroll
        for (int m = 0; m < 4 * KC; ++m) sacc[r][m] = 0.f;
    }
    if (a == b) {
        sob_sym_unit<KC, HILO, true>(A, a, b, lane, ms, Sh, Sl, Sn, aS, Su, sacc);
    } else {
        bool lo = HILO;
        if (HILO) {   // blocks far apart: the high parts suffice (tile_is_far)
            float4 ilo, ihi;
            irange_box(A.tbox, (int64_t)a * kSymFaces, kSymFaces, ilo, ihi);
            lo = false;
            for (int t = 0; t < kSymFaces / kTileJ; ++t)
                lo = lo || !tile_is_far(ilo, ihi, A.tbox, b * (kSymFaces / kTileJ) + t);
        }
        if (lo) sob_sym_unit<KC, HILO, false>(A, a, b, lane, ms, Sh, Sl, Sn, aS, Su, sacc);
        else sob_sym_unit<KC, false, false>(A, a, b, lane, ms, Sh, Sl, Sn, aS, Su, sacc);
    }
#pragma unroll
    for (int r = 0; r < kSymNI; ++r) {
        const int64_t S = (int64_t)(a - A.a0) * kSymFaces + r * 64 + lane;   // row in the band
#pragma unroll
        for (int m = 0; m < 4 * KC; ++m) A.partS[((int64_t)b * 4 * KC + m) * A.ldS + S] = sacc[r][m];
    }
}

// ------------------------------------------------------------------ FP64 pair sums

template <int KC>
__global__ __launch_bounds__(kBlock) void k_sob64(SobArgs A, double ms)
{
    const int bi = (int)blockIdx.x % A.n_itiles;
    const int bs = (int)blockIdx.x / A.n_itiles;
    const double4* __restrict__ dx4 = static_cast<const double4*>(A.fx);
    const double4* __restrict__ dn4 = static_cast<const double4*>(A.fn);
    const double4* __restrict__ fu = static_cast<const double4*>(A.fu);
    __shared__ double4 s_x[kTileJ], s_n[kTileJ], s_u[kTileJ * KC];
    const int64_t ibase = (int64_t)bi * kBlock;
    const int jt0 = bs * A.tiles_per_split;
    const int jt1 = min(jt0 + A.tiles_per_split, A.ntiles_j);
    const int64_t Si = ibase + threadIdx.x;
    const double4 x = dx4[Si], n = dn4[Si];
    double4 Su[KC];
    double acc[4 * KC];
#pragma unroll
    for (int cc = 0; cc < KC; ++cc) Su[cc] = fu[Si * KC + cc];
#pragma unroll
    for (int q = 0; q < 4 * KC; ++q) acc[q] = 0.0;
    for (int jt = jt0; jt < jt1; ++jt) {
        const int64_t j0 = (int64_t)jt * kTileJ;
        __syncthreads();
        for (int e = threadIdx.x; e < kTileJ; e += kBlock) {
            s_x[e] = dx4[j0 + e];
            s_n[e] = dn4[j0 + e];
        }
        for (int e = threadIdx.x; e < kTileJ * KC; e += kBlock) s_u[e] = fu[j0 * KC + e];
        __syncthreads();
        const bool diag = hits_diag(j0, ibase, kBlock);
        for (int jj = 0; jj < kTileJ; ++jj) {
            if (diag && Si == j0 + jj) continue;
            const double4 t = s_x[jj], tn = s_n[jj];
            const double dx = x.x - t.x, dy = x.y - t.y, dz = x.z - t.z;
            const double r2 = dx * dx + dy * dy + dz * dz;
            const double w = pow(r2, ms) * t.w;
            const double qs = n.x * dx + n.y * dy + n.z * dz;
            const double qt = tn.x * dx + tn.y * dy + tn.z * dz;
            const double w0 = w * (qs * qs + qt * qt) / (r2 * r2);
#pragma unroll
            for (int cc = 0; cc < KC; ++cc) {
                const double4 tu = s_u[jj * KC + cc];
                acc[4 * cc + 0] += w * (Su[cc].x - tu.x);
                acc[4 * cc + 1] += w * (Su[cc].y - tu.y);
                acc[4 * cc + 2] += w * (Su[cc].z - tu.z);
                acc[4 * cc + 3] += w0 * (Su[cc].w - tu.w);
            }
        }
    }
#pragma unroll
    for (int q = 0; q < 4 * KC; ++q) A.part[((int64_t)bs * 4 * KC + q) * A.irows + Si] = acc[q];
}

// ------------------------------------------------------------------ gather to vertices

__global__ void k_sob_gather(int64_t nV, const int32_t* __restrict__ vf_off, const int32_t* __restrict__ vf_idx,
                             const double* __restrict__ V, const int32_t* __restrict__ F,
                             const double4* __restrict__ dxa, const double* __restrict__ z, int64_t zs, int kc,
                             int ldo, int c0, double* __restrict__ Au)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nV * kc) return;
    const int64_t v = t / kc;
    const int c = (int)(t - v * kc);
    double acc = 0.0;
    for (int32_t q = vf_off[v]; q < vf_off[v + 1]; ++q) {
        const int64_t f = vf_idx[q] / 3;
        const int m = vf_idx[q] - 3 * (int)f;
        const double* pi = V + 3 * (int64_t)F[3 * f + m];
        const double* pj = V + 3 * (int64_t)F[3 * f + (m + 1) % 3];
        const double* pk = V + 3 * (int64_t)F[3 * f + (m + 2) % 3];
        const double e1[3] = {pj[0] - pi[0], pj[1] - pi[1], pj[2] - pi[2]};
        const double e2[3] = {pk[0] - pi[0], pk[1] - pi[1], pk[2] - pi[2]};
        const double cr[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2],
                              e1[0] * e2[1] - e1[1] * e2[0]};
        const double ic2 = 1.0 / (cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2]);
        const double e[3] = {pk[0] - pj[0], pk[1] - pj[1], pk[2] - pj[2]};
        const double g0 = (cr[1] * e[2] - cr[2] * e[1]) * ic2;
        const double g1 = (cr[2] * e[0] - cr[0] * e[2]) * ic2;
        const double g2 = (cr[0] * e[1] - cr[1] * e[0]) * ic2;
        const double* zc = z + (int64_t)(4 * c) * zs + f;
        acc += 2.0 * dxa[f].w * (g0 * zc[0] + g1 * zc[zs] + g2 * zc[2 * zs] + zc[3 * zs] / 6.0);
    }
    Au[v * ldo + c0 + c] = acc;
}

// Approximate diagonal of A from the row sums rs(S) = sum_T |d|^-2s a_T and
// r0(S) = sum_T |d|^-2s a_T (q_S^2 + q_T^2) / |d|^4 (z layout [4][irows]: rows 0 and 3):
//   diag_i = 2 sum_{S ni i} a_S (|D phi_i(S)|^2 rs(S) + r0(S) / 18),
// i.e. (A)_ii without the pairs S, T that both contain i (u = e_i has D u(T) = 0 and
// ubar(T) = 0 on every other face).  dinv = 1 / diag.
__global__ void k_sob_diag(int64_t nV, const int32_t* __restrict__ vf_off, const int32_t* __restrict__ vf_idx,
                           const double* __restrict__ V, const int32_t* __restrict__ F,
                           const double4* __restrict__ dxa, const double* __restrict__ z, int64_t zs,
                           double* __restrict__ dinv)
{
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= nV) return;
    double acc = 0.0;
    for (int32_t q = vf_off[v]; q < vf_off[v + 1]; ++q) {
        const int64_t f = vf_idx[q] / 3;
        const int m = vf_idx[q] - 3 * (int)f;
        const double* pi = V + 3 * (int64_t)F[3 * f + m];
        const double* pj = V + 3 * (int64_t)F[3 * f + (m + 1) % 3];
        const double* pk = V + 3 * (int64_t)F[3 * f + (m + 2) % 3];
        const double e1[3] = {pj[0] - pi[0], pj[1] - pi[1], pj[2] - pi[2]};
        const double e2[3] = {pk[0] - pi[0], pk[1] - pi[1], pk[2] - pi[2]};
        const double cr[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2],
                              e1[0] * e2[1] - e1[1] * e2[0]};
        const double c2 = cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2];
        const double e2n = (pk[0] - pj[0]) * (pk[0] - pj[0]) + (pk[1] - pj[1]) * (pk[1] - pj[1]) +
                           (pk[2] - pj[2]) * (pk[2] - pj[2]);
        // |c x e|^2 / |c|^4 = |e|^2 / |c|^2 (e lies in the face's plane, orthogonal to c)
        acc += 2.0 * dxa[f].w * (e2n / c2 * z[f] + z[3 * zs + f] / 18.0);
    }
    dinv[v] = acc > 0.0 ? 1.0 / acc : 0.0;
}

// ------------------------------------------------------------------ dispatch

const void* sob_fn(int precision, int kc)
{
    const bool hilo = precision == TP_PREC_FP32_HILO || precision == TP_PREC_FP32_NEAR64;
    if (precision == TP_PREC_FP64) {
        switch (kc) {
        case 1: return (const void*)k_sob64<1>;
        case 2: return (const void*)k_sob64<2>;
        default: return (const void*)k_sob64<3>;
        }
    }
    switch (kc) {
    case 1: return hilo ? (const void*)k_sob32<kNiSob32, 1, true> : (const void*)k_sob32<kNiSob32, 1, false>;
    case 2: return hilo ? (const void*)k_sob32<kNiSob32, 2, true> : (const void*)k_sob32<kNiSob32, 2, false>;
    default: return hilo ? (const void*)k_sob32<kNiSob32, 3, true> : (const void*)k_sob32<kNiSob32, 3, false>;
    }
}

int sob_occupancy(const void* fn)
{
    static std::mutex mu;
    static std::unordered_map<const void*, int> cache;
    std::lock_guard<std::mutex> lk(mu);
    auto it = cache.find(fn);
    if (it != cache.end()) return it->second;
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, kBlock, 0) != hipSuccess || nb < 1) nb = 1;
    cache[fn] = nb;
    return nb;
}

template <int KC>
void launch_pair_k(int precision, dim3 grid, const SobArgs& A, double sexp, hipStream_t st)
{
    const dim3 block(kBlock);
    if (precision == TP_PREC_FP64)
        hipLaunchKernelGGL(k_sob64<KC>, grid, block, 0, st, A, -sexp);
    else if (precision == TP_PREC_FP32_HILO || precision == TP_PREC_FP32_NEAR64)
        hipLaunchKernelGGL((k_sob32<kNiSob32, KC, true>), grid, block, 0, st, A, (float)-sexp);
    else
        hipLaunchKernelGGL((k_sob32<kNiSob32, KC, false>), grid, block, 0, st, A, (float)-sexp);
}

}  // namespace

PairPlan sobolev_plan(int precision, int kc, int64_t nF, int64_t cap)
{
    kc = std::max(1, std::min(kc, kSobCols));
    const int ni = precision == TP_PREC_FP64 ? 1 : kNiSob32;
    return plan_pairs(nF, cap, ni, sob_occupancy(sob_fn(precision, kc)));
}

size_t sobolev_face_bytes(int precision, int kc, int64_t cap)
{
    return (size_t)cap * (size_t)kc * (precision == TP_PREC_FP64 ? sizeof(double4) : sizeof(float4));
}

hipError_t launch_sobolev_diag(const SobolevCall& c, double* dinv, hipStream_t s)
{
    if (!c.fd) return hipErrorInvalidValue;
    const FaceData& fd = *c.fd;
    const PairPlan& pl = c.plan;
    if (pl.irows > fd.cap || (int64_t)pl.ntiles_j * kTileJ > fd.cap) return hipErrorInvalidValue;
    SobArgs A;
    A.fx = fd.fx;
    A.fl = fd.fl;
    A.fn = fd.fn;
    A.fu = nullptr;
    A.part = c.part;
    A.tbox = fd.tbox;
    A.irows = pl.irows;
    A.n_itiles = pl.n_itiles;
    A.tiles_per_split = pl.tiles_per_split;
    A.ntiles_j = pl.ntiles_j;
    const dim3 grid((unsigned)(pl.n_itiles * pl.n_split)), block(kBlock);
    // FP32 hi/lo pair terms whatever the problem's precision: the diagonal only preconditions
    hipLaunchKernelGGL((k_sob32<kNiSob32, 1, true, true>), grid, block, 0, s, A, (float)-c.s);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = launch_reduce_splits(c.part, pl.n_split, 4, pl.irows, c.nF, c.z, pl.irows, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_sob_diag, dim3(nblk(c.nV)), dim3(256), 0, s, c.nV, c.vf_off, c.vf_idx, c.V, c.F, fd.dx,
                       c.z, pl.irows, dinv);
    return hipGetLastError();
}

hipError_t launch_sobolev(const SobolevCall& c, const double* u, int ldu, int kc, double* Au, int ldo,
                          int c0, hipEvent_t ev0, hipEvent_t ev1, hipStream_t s)
{
    if (kc < 1 || kc > kSobCols || !c.fd) return hipErrorInvalidValue;
    const FaceData& fd = *c.fd;
    const PairPlan& pl = c.plan;
    // the kernels read faces [0, irows) and j-tiles [0, ntiles_j * kTileJ) of arrays of cap entries
    if (pl.irows > fd.cap || (int64_t)pl.ntiles_j * kTileJ > fd.cap) return hipErrorInvalidValue;
    const bool f64 = c.precision == TP_PREC_FP64;
    if (f64)
        hipLaunchKernelGGL((k_sob_face<double, double4>), dim3(nblk(fd.cap)), dim3(256), 0, s, c.V, c.F, c.nF,
                           fd.cap, u + c0, ldu, kc, static_cast<double4*>(c.fu));
    else
        hipLaunchKernelGGL((k_sob_face<float, float4>), dim3(nblk(fd.cap)), dim3(256), 0, s, c.V, c.F, c.nF,
                           fd.cap, u + c0, ldu, kc, static_cast<float4*>(c.fu));
    SobArgs A;
    A.fx = f64 ? (const void*)fd.dx : (const void*)fd.fx;
    A.fl = fd.fl;
    A.fn = f64 ? (const void*)fd.dn : (const void*)fd.fn;
    A.fu = c.fu;
    A.part = c.part;
    A.tbox = fd.tbox;
    A.irows = pl.irows;
    A.n_itiles = pl.n_itiles;
    A.tiles_per_split = pl.tiles_per_split;
    A.ntiles_j = pl.ntiles_j;
    if (c.symp) {
        if (f64 || c.sym_band < 1) return hipErrorInvalidValue;
        const bool hilo = c.precision == TP_PREC_FP32_HILO || c.precision == TP_PREC_FP32_NEAR64;
        SobSymArgs S;
        S.fx = fd.fx;
        S.fl = fd.fl;
        S.fn = fd.fn;
        S.fu = static_cast<const float4*>(c.fu);
        S.tbox = fd.tbox;
        S.nB = (int)((c.nF + kSymFaces - 1) / kSymFaces);
        const int K = std::min(c.sym_band, S.nB);
        sym_regions(c.symp, c.nF, 4 * kc, K, S.part, S.partS, S.ldp, S.ldS);
        // the blocks read faces [0, ldp) of arrays of cap entries
        if (S.ldp > fd.cap) return hipErrorInvalidValue;
        if (ev0) (void)hipEventRecord(ev0, s);
        for (int a0 = 0; a0 < S.nB; a0 += K) {
            S.a0 = a0;
            S.a1 = std::min(S.nB, a0 + K);
            const int64_t units = sym_band_units(c.nF, S.a0, S.a1);
            const dim3 grid((unsigned)((units + kBlock / 64 - 1) / (kBlock / 64)));
            const float ms = (float)-c.s;
            switch (kc) {
            case 1:
                if (hilo) hipLaunchKernelGGL((k_sob32_sym<1, true>), grid, dim3(kBlock), 0, s, S, ms);
                else hipLaunchKernelGGL((k_sob32_sym<1, false>), grid, dim3(kBlock), 0, s, S, ms);
                break;
            case 2:
                if (hilo) hipLaunchKernelGGL((k_sob32_sym<2, true>), grid, dim3(kBlock), 0, s, S, ms);
                else hipLaunchKernelGGL((k_sob32_sym<2, false>), grid, dim3(kBlock), 0, s, S, ms);
                break;
            default:
                if (hilo) hipLaunchKernelGGL((k_sob32_sym<3, true>), grid, dim3(kBlock), 0, s, S, ms);
                else hipLaunchKernelGGL((k_sob32_sym<3, false>), grid, dim3(kBlock), 0, s, S, ms);
                break;
            }
            if (ev1 && S.a1 == S.nB) (void)hipEventRecord(ev1, s);
            hipError_t e = hipGetLastError();
            if (e != hipSuccess) return e;
            e = launch_reduce_sym_band(c.symp, c.nF, 4 * kc, K, S.a0, S.a1, nullptr, c.z, pl.irows, s);
            if (e != hipSuccess) return e;
        }
        hipLaunchKernelGGL(k_sob_gather, dim3(nblk(c.nV * kc)), dim3(256), 0, s, c.nV, c.vf_off, c.vf_idx, c.V, c.F,
                           fd.dx, c.z, pl.irows, kc, ldo, c0, Au);
        return hipGetLastError();
    }
    const dim3 grid((unsigned)(pl.n_itiles * pl.n_split));
    if (ev0) (void)hipEventRecord(ev0, s);
    switch (kc) {
    case 1: launch_pair_k<1>(c.precision, grid, A, c.s, s); break;
    case 2: launch_pair_k<2>(c.precision, grid, A, c.s, s); break;
    default: launch_pair_k<3>(c.precision, grid, A, c.s, s); break;
    }
    if (ev1) (void)hipEventRecord(ev1, s);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = launch_reduce_splits(c.part, pl.n_split, 4 * kc, pl.irows, c.nF, c.z, pl.irows, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_sob_gather, dim3(nblk(c.nV * kc)), dim3(256), 0, s, c.nV, c.vf_off, c.vf_idx, c.V, c.F,
                       fd.dx, c.z, pl.irows, kc, ldo, c0, Au);
    return hipGetLastError();
}

// ------------------------------------------------------------------ Krylov vectors

namespace {

constexpr int kKryBlocks = 256;   // workgroups of the first reduction stage
constexpr int kKryMaxOut = 1024;  // outputs of one krylov_dots call (nvec * k)

__global__ __launch_bounds__(256) void k_kry_dots(const double* __restrict__ Vb, int64_t vstride, int nvec,
                                                  const double* __restrict__ w, int64_t n, int k,
                                                  double* __restrict__ partial)
{
    // rows [b, e) of this workgroup; one thread per (row, column) element of the chunk
    __shared__ double sh[4];
    const int64_t chunk = (n + kKryBlocks - 1) / kKryBlocks;
    const int64_t b = (int64_t)blockIdx.x * chunk, e = min(n, b + chunk);
    const int m = nvec * k;
    for (int o = 0; o < m; ++o) {
        const int i = o / k, c = o - i * k;
        const double* V = Vb + (int64_t)i * vstride;
        double acc = 0.0;
        for (int64_t r = b + threadIdx.x; r < e; r += 256) acc += V[r * k + c] * w[r * k + c];
        for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
        if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
        __syncthreads();
        if (threadIdx.x == 0) partial[(int64_t)blockIdx.x * m + o] = (sh[0] + sh[1]) + (sh[2] + sh[3]);
        __syncthreads();
    }
}

__global__ void k_kry_final(const double* __restrict__ partial, int m, double* __restrict__ out)
{
    const int o = blockIdx.x * blockDim.x + threadIdx.x;
    if (o >= m) return;
    double acc = 0.0;
    for (int q = 0; q < kKryBlocks; ++q) acc += partial[(int64_t)q * m + o];
    out[o] = acc;
}

__global__ void k_kry_subtract(double* __restrict__ w, const double* __restrict__ Vb, int64_t vstride, int nvec,
                               const double* __restrict__ h, int64_t n, int k)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * k) return;
    const int c = (int)(t % k);
    double acc = w[t];
    for (int i = 0; i < nvec; ++i) acc -= h[i * k + c] * Vb[(int64_t)i * vstride + t];
    w[t] = acc;
}

__global__ void k_kry_combine(double* __restrict__ x, const double* __restrict__ Zb, int64_t vstride, int nvec,
                              const double* __restrict__ y, int64_t n, int k, int accumulate)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * k) return;
    const int c = (int)(t % k);
    double acc = accumulate ? x[t] : 0.0;
    for (int i = 0; i < nvec; ++i) acc += y[i * k + c] * Zb[(int64_t)i * vstride + t];
    x[t] = acc;
}

__global__ void k_kry_scale(double* __restrict__ dst, const double* __restrict__ src,
                            const double* __restrict__ scale, int64_t n, int k)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * k) return;
    dst[t] = src[t] * scale[t % k];
}

__global__ void k_kry_diag_add(double* __restrict__ Z, const double* __restrict__ V,
                               const double* __restrict__ dinv, double omega, int64_t n, int k)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * k) return;
    Z[t] += omega * dinv[t / k] * V[t];
}

__global__ void k_kry_indicators(const int32_t* __restrict__ label, int64_t n, int nl, int width,
                                 double* __restrict__ out)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t per = n * width;
    if (t >= per * nl) return;
    const int64_t l = t / per;
    const int64_t v = (t - l * per) / width;
    out[t] = label[v] == (int32_t)l ? 1.0 : 0.0;
}

}  // namespace

hipError_t krylov_diag_add(double* Z, const double* V, const double* dinv, double omega, int64_t n, int k,
                           hipStream_t s)
{
    hipLaunchKernelGGL(k_kry_diag_add, dim3(nblk(n * k)), dim3(256), 0, s, Z, V, dinv, omega, n, k);
    return hipGetLastError();
}

hipError_t krylov_indicators(const int32_t* label, int64_t n, int nl, int width, double* out, hipStream_t s)
{
    hipLaunchKernelGGL(k_kry_indicators, dim3(nblk(n * width * nl)), dim3(256), 0, s, label, n, nl, width, out);
    return hipGetLastError();
}

size_t krylov_scratch_doubles(int m) { return (size_t)kKryBlocks * (size_t)std::max(1, m); }

hipError_t krylov_dots(const double* Vb, int64_t vstride, int nvec, const double* w, int64_t n, int k,
                       double* scratch, double* out, hipStream_t s)
{
    const int m = nvec * k;
    if (nvec < 1 || k < 1 || m > kKryMaxOut) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_kry_dots, dim3(kKryBlocks), dim3(256), 0, s, Vb, vstride, nvec, w, n, k, scratch);
    hipLaunchKernelGGL(k_kry_final, dim3(nblk(m)), dim3(256), 0, s, scratch, m, out);
    return hipGetLastError();
}

hipError_t krylov_subtract(double* w, const double* Vb, int64_t vstride, int nvec, const double* h, int64_t n,
                           int k, hipStream_t s)
{
    hipLaunchKernelGGL(k_kry_subtract, dim3(nblk(n * k)), dim3(256), 0, s, w, Vb, vstride, nvec, h, n, k);
    return hipGetLastError();
}

hipError_t krylov_combine(double* x, const double* Zb, int64_t vstride, int nvec, const double* y, int64_t n,
                          int k, bool accumulate, hipStream_t s)
{
    hipLaunchKernelGGL(k_kry_combine, dim3(nblk(n * k)), dim3(256), 0, s, x, Zb, vstride, nvec, y, n, k,
                       accumulate ? 1 : 0);
    return hipGetLastError();
}

hipError_t krylov_scale(double* dst, const double* src, const double* scale, int64_t n, int k, hipStream_t s)
{
    hipLaunchKernelGGL(k_kry_scale, dim3(nblk(n * k)), dim3(256), 0, s, dst, src, scale, n, k);
    return hipGetLastError();
}

}  // namespace tp
