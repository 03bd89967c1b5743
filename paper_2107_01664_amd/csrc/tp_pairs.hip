// All-pairs face-face kernels of the tangent-point hot path (gfx950).
//
// Two shapes.  The symmetric kernels (k_grad32_sym, k_frac32_sym, k_energy32_sym, from
// 16,384 faces on) evaluate each unordered pair once for both rows: one wave per pair of
// 256-face blocks, faces T passed along the wave (see their section below).  The row-by-row
// kernels (k_*32, k_*64, the FP64 near field) evaluate every ordered pair for its row: a
// workgroup owns an i-tile of kBlock * NI faces S
// held in registers (NI per thread) and streams a contiguous range of j-tiles of kTileJ
// faces T through LDS; every lane reads the same T (LDS broadcast).  Each problem's
// workgroups form an (i-tiles) x (j-splits) grid; one launch concatenates the grids of up
// to kMaxPairJobs problems (same-phase work of several meshes in one launch).  Each
// workgroup writes its per-face sums for its j-range to a partial buffer, and a separate
// pass adds the splits in order, so results do not depend on scheduling or on the other
// problems of the launch.  The diagonal S = T is excluded by forcing |d|^2 = 1 where d = 0, which
// makes every term vanish; only tiles that intersect the i-range take that check.
//
// Arithmetic (FP32 variants): pair terms in FP32 on the vector ALUs, per-tile sums in
// FP32 over kTileJ terms, then added into FP64 accumulators.  With HILO the barycenter
// difference is formed as (Xhi_S - Xhi_T) + (Xlo_S - Xlo_T) from an FP32 hi/lo split of
// the FP64 barycenter, which keeps d accurate for near pairs (the kernel raises q = N.d
// to the 6th power, and q is small for near pairs on a smooth surface); tiles far from
// the i-range (tile_is_far) use the high parts alone.
#include "tp_internal.h"
#include "tp_sym.h"
#include "tp_tiles.h"

#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <unordered_map>
#include <vector>

namespace tp {

// ------------------------------------------------------------------ fast math helpers

__device__ __forceinline__ float rcp_fast(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double rcp_fast(double x)
{
    double y = __builtin_amdgcn_rcp(x);       // v_rcp_f64, refined by two Newton steps
    double e = __builtin_fma(-x, y, 1.0);
    y = __builtin_fma(y, e, y);
    e = __builtin_fma(-x, y, 1.0);
    return __builtin_fma(y, e, y);
}
__device__ __forceinline__ float log2_fast(float x) { return __builtin_amdgcn_logf(x); }
__device__ __forceinline__ float exp2_fast(float x) { return __builtin_amdgcn_exp2f(x); }

// ------------------------------------------------------------------ exponent policies
//
// Kernel of eq. DiscreteTangentPointKernel with q = N_S . d, r2 = |d|^2:
//   K   = |q|^alpha r2^(-beta/2)
//   Kqr = K r2 / q = sgn(q) |q|^(alpha-1) r2^(1 - beta/2)   (0 when q = 0, alpha > 1)
// so that dK/dd = alpha (Kqr / r2) N_S - beta (K / r2) d  and  dK/dN_S = alpha (Kqr / r2) d.

// alpha = 6, beta = 12 (p = 6, Sec. 2.1): with u = q / r2, K = u^6 and Kqr = u^5.
struct PowP6 {
    template <class R>
    __device__ __forceinline__ R K(R q, R r2, R inv) const
    {
        (void)r2;
        R u = q * inv;
        R u2 = u * u;
        return u2 * u2 * u2;
    }
    template <class R>
    __device__ __forceinline__ void KG(R q, R r2, R inv, R& K, R& Kqr) const
    {
        (void)r2;
        R u = q * inv;
        R u2 = u * u;
        R u4 = u2 * u2;
        K = u4 * u2;
        Kqr = u4 * u;
    }
};

// General exponents through log2 / exp2, written on u = q / r2 (the same quantity the
// p = 6 policy raises to integer powers):
//   K = |u|^alpha r2^gamma,   Kqr = sgn(q) |u|^(alpha-1) r2^gamma,   gamma = alpha - beta/2.
// The FP32 exponent (alpha-1) log2|u| + gamma log2 r2 then stays small: |u| is of the order
// of the curvature and gamma is zero for beta = 2 alpha.  Written on q and r2 separately,
// the two logarithms are each tens of units and cancel, and the FP32 rounding of those
// terms becomes a relative error of K several times larger.
struct PowGen {
    float am1;      // alpha - 1
    float gam;      // alpha - beta / 2
    double am1d, hbd;
    __device__ __forceinline__ float K(float q, float r2, float inv) const
    {
        if (r2 == INFINITY) return 0.0f;   // a pair left out of the FP32 sums
        const float lu = log2_fast(fabsf(q * inv));
        const float e = (am1 + 1.0f) * lu + (gam != 0.0f ? gam * log2_fast(r2) : 0.0f);
        return exp2_fast(e);
    }
    __device__ __forceinline__ void KG(float q, float r2, float inv, float& K, float& Kqr) const
    {
        if (r2 == INFINITY) {      // a pair left out of the FP32 sums
            K = 0.0f;
            Kqr = 0.0f;
            return;
        }
        const float u = q * inv;
        const float e = am1 * log2_fast(fabsf(u)) + (gam != 0.0f ? gam * log2_fast(r2) : 0.0f);
        Kqr = copysignf(exp2_fast(e), q);
        K = Kqr * u;
    }
    __device__ __forceinline__ double K(double q, double r2, double inv) const
    {
        (void)inv;
        return pow(fabs(q), am1d + 1.0) * pow(r2, -hbd);
    }
    __device__ __forceinline__ void KG(double q, double r2, double inv, double& K, double& Kqr) const
    {
        Kqr = copysign(pow(fabs(q), am1d) * pow(r2, 1.0 - hbd), q);
        K = Kqr * q * inv;
    }
};

// ------------------------------------------------------------------ job selection

struct PairBatch {
    PairJob j[kMaxPairJobs];
    int n;
};

// The job of this workgroup: the last one whose first workgroup is at or below blockIdx.x.
// Every index is a compile-time constant and every condition is uniform, so the selection
// stays in scalar registers.
__device__ __forceinline__ PairJob pick_job(const PairBatch& jb)
{
    PairJob J = jb.j[0];
    const int b = blockIdx.x;
#pragma unroll
    for (int q = 1; q < kMaxPairJobs; ++q)
        if (q < jb.n && b >= jb.j[q].block0) J = jb.j[q];
    return J;
}

// ------------------------------------------------------------------ tile loading

template <bool HILO>
__device__ __forceinline__ void load_tile3(const float4* __restrict__ fx, const float4* __restrict__ fl,
                                           const float4* __restrict__ fn, float4* s_x, float4* s_l,
                                           float4* s_n, int64_t j0)
{
    constexpr int parts = HILO ? 3 : 2;
    for (int e = threadIdx.x; e < parts * kTileJ; e += kBlock) {
        int w = e / kTileJ, jj = e - w * kTileJ;
        if (w == 0) s_x[jj] = fx[j0 + jj];
        else if (w == 1) s_n[jj] = fn[j0 + jj];
        else s_l[jj] = fl[j0 + jj];
    }
}

__device__ __forceinline__ bool tile_hits_diag(int64_t j0, int64_t ibase, int ispan)
{
    return j0 < ibase + ispan && j0 + kTileJ > ibase;
}

// Can a pair of the i-range box and j-tile jt be closer than the near-field radius?  The
// boxes hold the FP32 barycenters, within rounding of the hi+lo distances, so the test
// uses a 1 % margin.
__device__ __forceinline__ bool tile_may_be_near(const float4& ilo, const float4& ihi, const float4* tbox,
                                                 int jt, float rho2)
{
    const float4 a = tbox[2 * jt], b = tbox[2 * jt + 1];
    const float gx = fmaxf(fmaxf(a.x - ihi.x, ilo.x - b.x), 0.f);
    const float gy = fmaxf(fmaxf(a.y - ihi.y, ilo.y - b.y), 0.f);
    const float gz = fmaxf(fmaxf(a.z - ihi.z, ilo.z - b.z), 0.f);
    return gx * gx + gy * gy + gz * gz <= 1.01f * rho2;
}

// ------------------------------------------------------------------ per-face accumulators
//
// What a face's running sum over the j-tiles of its split is kept in: FP64 (the library's
// arithmetic), or, for the precision sweep only, plain FP32 or FP32 with Kahan's
// compensated summation.  Each j-tile's 128 terms are summed in FP32 in every case; the
// sums over splits, the chain rule to vertices and the energy total stay FP64.
enum { kAcc64 = 0, kAcc32 = 1, kAccKahan = 2 };

template <int ACC> struct FaceAcc;
template <> struct FaceAcc<kAcc64> {
    double s;
    __device__ __forceinline__ void clear() { s = 0.0; }
    __device__ __forceinline__ void add(float c) { s += (double)c; }
    __device__ __forceinline__ double value() const { return s; }
};
template <> struct FaceAcc<kAcc32> {
    float s;
    __device__ __forceinline__ void clear() { s = 0.f; }
    __device__ __forceinline__ void add(float c) { s += c; }
    __device__ __forceinline__ double value() const { return (double)s; }
};
template <> struct FaceAcc<kAccKahan> {
    float s, e;   // sum and the running error of its last additions (Kahan 1965)
    __device__ __forceinline__ void clear() { s = 0.f; e = 0.f; }
    __device__ __forceinline__ void add(float c)
    {
        const float y = c - e;
        const float t = s + y;
        e = (t - s) - y;
        s = t;
    }
    __device__ __forceinline__ double value() const { return (double)s; }
};

// ============================================================== energy (FP32)

// Squared FP32 distance of a pair, in one fixed sequence of operations (the FP64 near
// field repeats it bit for bit to decide which pairs it owns).
__device__ __forceinline__ float dist2_32(float dx, float dy, float dz)
{
    return __builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, dx * dx));
}

template <bool DIAG, int NI, bool HILO, bool NEAR, class Pow>
__device__ __forceinline__ void energy_tile32(const float4* s_x, const float4* s_l, int64_t j0,
                                              const float3 (&Sh)[NI], const float3 (&Sl)[NI],
                                              const float3 (&Sn)[NI], const int64_t (&Si)[NI],
                                              const Pow& pw, float rho2, float (&c)[NI])
{
#pragma unroll 4
    for (int jj = 0; jj < kTileJ; ++jj) {
        const float4 tx = s_x[jj];
        float4 tl = make_float4(0.f, 0.f, 0.f, 0.f);
        if (HILO) tl = s_l[jj];
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
            float r2 = dist2_32(dx, dy, dz);
            if (DIAG) r2 = (Si[r] == j0 + jj) ? 1.0f : r2;
            if (NEAR) r2 = r2 < rho2 ? INFINITY : r2;   // summed by the FP64 near field
            const float inv = rcp_fast(r2);
            const float q = Sn[r].x * dx + Sn[r].y * dy + Sn[r].z * dz;
            c[r] += pw.K(q, r2, inv) * tx.w;
        }
    }
}

template <int NI, bool HILO, bool NEAR, class Pow, int ACC = kAcc64>
__global__ __launch_bounds__(kBlock) void k_energy32(PairBatch jb, Pow pw)
{
    const PairJob J = pick_job(jb);
    const int bi = ((int)blockIdx.x - J.block0) % J.n_itiles;
    const int bs = ((int)blockIdx.x - J.block0) / J.n_itiles;
    const int tiles_per_split = J.tiles_per_split, ntiles_j = J.ntiles_j;
    double* __restrict__ part = J.part;
    const int64_t irows = J.irows;
    const float4* __restrict__ fx = J.fx;
    const float4* __restrict__ fl = J.fl;
    const float4* __restrict__ fn = J.fn;
    __shared__ float4 s_x[kTileJ], s_l[HILO ? kTileJ : 1], s_n[kTileJ];
    const int64_t ibase = (int64_t)bi * (kBlock * NI);
    const int jt0 = bs * tiles_per_split;
    const int jt1 = min(jt0 + tiles_per_split, ntiles_j);
    float3 Sh[NI], Sl[NI], Sn[NI];
    int64_t Si[NI];
    FaceAcc<ACC> acc[NI];
#pragma unroll
    for (int r = 0; r < NI; ++r) {
        Si[r] = ibase + r * kBlock + threadIdx.x;
        float4 x = fx[Si[r]], n = fn[Si[r]];
        Sh[r] = make_float3(x.x, x.y, x.z);
        Sn[r] = make_float3(n.x, n.y, n.z);
        if (HILO) {
            float4 l = fl[Si[r]];
            Sl[r] = make_float3(l.x, l.y, l.z);
        } else {
            Sl[r] = make_float3(0.f, 0.f, 0.f);
        }
        acc[r].clear();
    }
    float4 ilo, ihi;
    if (NEAR || HILO) irange_box(J.tbox, ibase, kBlock * NI, ilo, ihi);
    for (int jt = jt0; jt < jt1; ++jt) {
        const int64_t j0 = (int64_t)jt * kTileJ;
        __syncthreads();
        load_tile3<HILO>(fx, fl, fn, s_x, s_l, s_n, j0);
        __syncthreads();
        float c[NI];
#pragma unroll
        for (int r = 0; r < NI; ++r) c[r] = 0.f;
        if (tile_hits_diag(j0, ibase, kBlock * NI))
            energy_tile32<true, NI, HILO, NEAR>(s_x, s_l, j0, Sh, Sl, Sn, Si, pw, J.rho2, c);
        else if (NEAR && tile_may_be_near(ilo, ihi, J.tbox, jt, J.rho2))
            energy_tile32<false, NI, HILO, NEAR>(s_x, s_l, j0, Sh, Sl, Sn, Si, pw, J.rho2, c);
        else if (HILO && tile_is_far(ilo, ihi, J.tbox, jt))
            energy_tile32<false, NI, false, false>(s_x, s_l, j0, Sh, Sl, Sn, Si, pw, J.rho2, c);
        else
            energy_tile32<false, NI, HILO, false>(s_x, s_l, j0, Sh, Sl, Sn, Si, pw, J.rho2, c);
#pragma unroll
        for (int r = 0; r < NI; ++r) acc[r].add(c[r]);
    }
#pragma unroll
    for (int r = 0; r < NI; ++r) part[(int64_t)bs * irows + Si[r]] = acc[r].value();
}

// ============================================================== energy + differential (FP32)
//
// Row ownership: face S collects every partial derivative with respect to its own
// quantities, from the pairs (S,T) and (T,S) (both share d, r2 and 1/r2):
//   dE/dX_S = a_S sum_T a_T [alpha (K/q) N_S + alpha (K'/q') N_T - beta (K + K') d / r2]
//   dE/dN_S = a_S sum_T a_T alpha (K/q) d
//   dE/da_S =     sum_T a_T (K + K')
// with d = X_S - X_T, q = N_S.d, q' = N_T.d, K = K(S,T), K' = K(T,S).  The per-tile
// accumulators c[0..10] are
//   c0 = sum a_T K/q,  c1..3 = sum a_T (K'/q') N_T,  c4..6 = sum a_T (K+K')/r2 d,
//   c7..9 = sum a_T (K/q) d,  c10 = sum a_T (K + K').
constexpr int kGradAcc = 11;
constexpr int kGradOut = 7;     // dE/dX (3), dE/dN (3), dE/da (1)

template <bool DIAG, int NI, bool HILO, bool NEAR, class Pow>
__device__ __forceinline__ void grad_tile32(const float4* s_x, const float4* s_l, const float4* s_n,
                                            int64_t j0, const float3 (&Sh)[NI],
                                            const float3 (&Sl)[NI], const float3 (&Sn)[NI],
                                            const int64_t (&Si)[NI], const Pow& pw, float rho2,
                                            float (&c)[NI][kGradAcc])
{
#pragma unroll 2
    for (int jj = 0; jj < kTileJ; ++jj) {
        const float4 tx = s_x[jj];
        const float4 tn = s_n[jj];
        float4 tl = make_float4(0.f, 0.f, 0.f, 0.f);
        if (HILO) tl = s_l[jj];
        const float aT = tx.w;
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
            float r2 = dist2_32(dx, dy, dz);
            if (DIAG) r2 = (Si[r] == j0 + jj) ? 1.0f : r2;
            if (NEAR) r2 = r2 < rho2 ? INFINITY : r2;   // summed by the FP64 near field
            const float inv = rcp_fast(r2);
            const float q = Sn[r].x * dx + Sn[r].y * dy + Sn[r].z * dz;
            const float qp = tn.x * dx + tn.y * dy + tn.z * dz;
            float K, Kqr, Kp, Kpqr;
            pw.KG(q, r2, inv, K, Kqr);
            pw.KG(qp, r2, inv, Kp, Kpqr);
            const float t = aT * inv;
            const float aq = Kqr * t;
            const float ap = Kpqr * t;
            const float KK = K + Kp;
            const float cc = KK * t;
            c[r][0] += aq;
            c[r][1] += ap * tn.x;
            c[r][2] += ap * tn.y;
            c[r][3] += ap * tn.z;
            c[r][4] += cc * dx;
            c[r][5] += cc * dy;
            c[r][6] += cc * dz;
            c[r][7] += aq * dx;
            c[r][8] += aq * dy;
            c[r][9] += aq * dz;
            c[r][10] += KK * aT;
        }
    }
}

template <int NI, bool HILO, bool NEAR, class Pow, int ACC = kAcc64>
__global__ __launch_bounds__(kBlock) void k_grad32(PairBatch jb, double alpha, double beta, Pow pw)
{
    const PairJob J = pick_job(jb);
    const int bi = ((int)blockIdx.x - J.block0) % J.n_itiles;
    const int bs = ((int)blockIdx.x - J.block0) / J.n_itiles;
    const int tiles_per_split = J.tiles_per_split, ntiles_j = J.ntiles_j;
    double* __restrict__ part = J.part;
    const int64_t irows = J.irows;
    const float4* __restrict__ fx = J.fx;
    const float4* __restrict__ fl = J.fl;
    const float4* __restrict__ fn = J.fn;
    const double4* __restrict__ dxa = J.dx;
    const double4* __restrict__ dn = J.dn;
    __shared__ float4 s_x[kTileJ], s_l[HILO ? kTileJ : 1], s_n[kTileJ];
    const int64_t ibase = (int64_t)bi * (kBlock * NI);
    const int jt0 = bs * tiles_per_split;
    const int jt1 = min(jt0 + tiles_per_split, ntiles_j);
    float3 Sh[NI], Sl[NI], Sn[NI];
    int64_t Si[NI];
    FaceAcc<ACC> acc[NI][kGradAcc];
#pragma unroll
    for (int r = 0; r < NI; ++r) {
        Si[r] = ibase + r * kBlock + threadIdx.x;
        float4 x = fx[Si[r]], n = fn[Si[r]];
        Sh[r] = make_float3(x.x, x.y, x.z);
        Sn[r] = make_float3(n.x, n.y, n.z);
        if (HILO) {
            float4 l = fl[Si[r]];
            Sl[r] = make_float3(l.x, l.y, l.z);
        } else {
            Sl[r] = make_float3(0.f, 0.f, 0.f);
        }
#pragma unroll
        for (int m = 0; m < kGradAcc; ++m) acc[r][m].clear();
    }
    float4 ilo, ihi;
    if (NEAR || HILO) irange_box(J.tbox, ibase, kBlock * NI, ilo, ihi);
    for (int jt = jt0; jt < jt1; ++jt) {
        const int64_t j0 = (int64_t)jt * kTileJ;
        __syncthreads();
        load_tile3<HILO>(fx, fl, fn, s_x, s_l, s_n, j0);
        __syncthreads();
        float c[NI][kGradAcc];
#pragma unroll
        for (int r = 0; r < NI; ++r)
#pragma unroll
            for (int m = 0; m < kGradAcc; ++m) c[r][m] = 0.f;
        if (tile_hits_diag(j0, ibase, kBlock * NI))
            grad_tile32<true, NI, HILO, NEAR>(s_x, s_l, s_n, j0, Sh, Sl, Sn, Si, pw, J.rho2, c);
        else if (NEAR && tile_may_be_near(ilo, ihi, J.tbox, jt, J.rho2))
            grad_tile32<false, NI, HILO, NEAR>(s_x, s_l, s_n, j0, Sh, Sl, Sn, Si, pw, J.rho2, c);
        else if (HILO && tile_is_far(ilo, ihi, J.tbox, jt))
            grad_tile32<false, NI, false, false>(s_x, s_l, s_n, j0, Sh, Sl, Sn, Si, pw, J.rho2, c);
        else
            grad_tile32<false, NI, HILO, false>(s_x, s_l, s_n, j0, Sh, Sl, Sn, Si, pw, J.rho2, c);
#pragma unroll
        for (int r = 0; r < NI; ++r)
#pragma unroll
            for (int m = 0; m < kGradAcc; ++m) acc[r][m].add(c[r][m]);
    }
#pragma unroll
    for (int r = 0; r < NI; ++r) {
        const double aS = dxa[Si[r]].w;
        const double4 N = dn[Si[r]];
        double a[kGradAcc];
#pragma unroll
        for (int m = 0; m < kGradAcc; ++m) a[m] = acc[r][m].value();
        double out[kGradOut];
        out[0] = aS * (alpha * (N.x * a[0] + a[1]) - beta * a[4]);
        out[1] = aS * (alpha * (N.y * a[0] + a[2]) - beta * a[5]);
        out[2] = aS * (alpha * (N.z * a[0] + a[3]) - beta * a[6]);
        out[3] = aS * alpha * a[7];
        out[4] = aS * alpha * a[8];
        out[5] = aS * alpha * a[9];
        out[6] = a[10];
        double* dst = part + (int64_t)bs * kGradOut * irows + Si[r];
#pragma unroll
        for (int m = 0; m < kGradOut; ++m) dst[m * irows] = out[m];
    }
}

// ============================================================== fractional apply (FP32)
//
// z(S) = sum_{T != S} |X_S - X_T|^-(2 sigma + 2) a_T (ubar_S - ubar_T)  for KC columns,
// the row sum of [diag(diag(a)^-1 H a) - H] U u divided by a_S (Sec. 5.1.1, App. A); the
// remaining factors 2 U^T diag(a) are applied per vertex afterwards.  Differences of the
// face averages are taken per pair, so no large cancelling sums are formed.
template <int KC>
struct KPad { static constexpr int value = (KC + 3) / 4 * 4; };

template <bool DIAG, int NI, int KC, bool HILO>
__device__ __forceinline__ void frac_tile32(const float4* s_x, const float4* s_l, const float* s_u,
                                            int64_t j0, const float3 (&Sh)[NI],
                                            const float3 (&Sl)[NI], const float (&Su)[NI][KC],
                                            const int64_t (&Si)[NI], float expo,
                                            float (&c)[NI][KC])
{
    constexpr int KP = KPad<KC>::value;
#pragma unroll 2
    for (int jj = 0; jj < kTileJ; ++jj) {
        const float4 tx = s_x[jj];
        float4 tl = make_float4(0.f, 0.f, 0.f, 0.f);
        if (HILO) tl = s_l[jj];
        float tu[KP];
#pragma unroll
        for (int q = 0; q < KP / 4; ++q) {
            float4 v = reinterpret_cast<const float4*>(s_u + jj * KP)[q];
            tu[4 * q] = v.x; tu[4 * q + 1] = v.y; tu[4 * q + 2] = v.z; tu[4 * q + 3] = v.w;
        }
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
            const float w = exp2_fast(expo * log2_fast(r2)) * tx.w;
#pragma unroll
            for (int cc = 0; cc < KC; ++cc) c[r][cc] += w * (Su[r][cc] - tu[cc]);
        }
    }
}

template <int NI, int KC, bool HILO>
__global__ __launch_bounds__(kBlock) void k_frac32(PairBatch jb, float expo)
{
    const PairJob J = pick_job(jb);
    const int bi = ((int)blockIdx.x - J.block0) % J.n_itiles;
    const int bs = ((int)blockIdx.x - J.block0) / J.n_itiles;
    const int tiles_per_split = J.tiles_per_split, ntiles_j = J.ntiles_j;
    double* __restrict__ part = J.part;
    const int64_t irows = J.irows;
    const float4* __restrict__ fx = J.fx;
    const float4* __restrict__ fl = J.fl;
    const float* __restrict__ ub = static_cast<const float*>(J.ub);
    constexpr int KP = KPad<KC>::value;
    __shared__ float4 s_x[kTileJ], s_l[HILO ? kTileJ : 1];
    __shared__ __align__(16) float s_u[kTileJ * KP];
    const int64_t ibase = (int64_t)bi * (kBlock * NI);
    const int jt0 = bs * tiles_per_split;
    const int jt1 = min(jt0 + tiles_per_split, ntiles_j);
    float3 Sh[NI], Sl[NI];
    float Su[NI][KC];
    int64_t Si[NI];
    double acc[NI][KC];
#pragma unroll
    for (int r = 0; r < NI; ++r) {
        Si[r] = ibase + r * kBlock + threadIdx.x;
        float4 x = fx[Si[r]];
        Sh[r] = make_float3(x.x, x.y, x.z);
        if (HILO) {
            float4 l = fl[Si[r]];
            Sl[r] = make_float3(l.x, l.y, l.z);
        } else {
            Sl[r] = make_float3(0.f, 0.f, 0.f);
        }
#pragma unroll
        for (int cc = 0; cc < KC; ++cc) {
            Su[r][cc] = ub[Si[r] * KP + cc];
            acc[r][cc] = 0.0;
        }
    }
    float4 ilo, ihi;
    if (HILO) irange_box(J.tbox, ibase, kBlock * NI, ilo, ihi);
    for (int jt = jt0; jt < jt1; ++jt) {
        const int64_t j0 = (int64_t)jt * kTileJ;
        __syncthreads();
        for (int e = threadIdx.x; e < kTileJ; e += kBlock) {
            s_x[e] = fx[j0 + e];
            if (HILO) s_l[e] = fl[j0 + e];
        }
        for (int e = threadIdx.x; e < kTileJ * KP / 4; e += kBlock)
            reinterpret_cast<float4*>(s_u)[e] = reinterpret_cast<const float4*>(ub + j0 * KP)[e];
        __syncthreads();
        float c[NI][KC];
#pragma unroll
        for (int r = 0; r < NI; ++r)
#pragma unroll
            for (int cc = 0; cc < KC; ++cc) c[r][cc] = 0.f;
        if (tile_hits_diag(j0, ibase, kBlock * NI))
            frac_tile32<true, NI, KC, HILO>(s_x, s_l, s_u, j0, Sh, Sl, Su, Si, expo, c);
        else if (HILO && tile_is_far(ilo, ihi, J.tbox, jt))
            frac_tile32<false, NI, KC, false>(s_x, s_l, s_u, j0, Sh, Sl, Su, Si, expo, c);
        else
            frac_tile32<false, NI, KC, HILO>(s_x, s_l, s_u, j0, Sh, Sl, Su, Si, expo, c);
#pragma unroll
        for (int r = 0; r < NI; ++r)
#pragma unroll
            for (int cc = 0; cc < KC; ++cc) acc[r][cc] += (double)c[r][cc];
    }
#pragma unroll
    for (int r = 0; r < NI; ++r)
#pragma unroll
        for (int cc = 0; cc < KC; ++cc)
            part[((int64_t)bs * KC + cc) * irows + Si[r]] = acc[r][cc];
}

// ============================================================== symmetric fractional apply (FP32)
//
// The kernel matrix of L^sigma is symmetric up to the areas: the (T,S) term of row T is
// g a_S (u_T - u_S) with the same g = r2^expo as the (S,T) term g a_T (u_S - u_T) of row S
// (and the FP32 difference X_T - X_S is exactly the negated X_S - X_T, so g is the same
// bits).  Here every unordered pair is evaluated once and adds to both rows.  Faces are
// cut into blocks of kSymFaces; a wave takes one pair of blocks (a, b), b >= a: its 64
// lanes hold the kSymNI faces S of block a each, and the faces T of block b pass along the
// wave 64 at a time, one lane a step (a rotation of the whole wave), carrying their own column
// sums.  For b > a both rows collect; the diagonal blocks (b = a) are summed row by row
// (S-side only, S = T left out), as in k_frac32.  A wave writes its S-side sums to slice b
// and its T-side sums to slice a of FP32 partial buffers: every face gets each slice exactly
// once (slices >= its block from its own rows, slices < its block from the waves in which it
// was T), and k_reduce_sym_band adds them in slice order in FP64.  A launch covers the rows a
// of one band [a0, a1); slice a of row T's sums is stored at a - a0 ([K][kc][ldp]) and row
// S's sums for the band's faces in [nB][kc][ldS], so the buffers grow with the band height K,
// not with nB, and the reductions of successive bands add the slices in the same order.

template <int KC, bool LO, bool DIAG>
__device__ __forceinline__ void sym_unit(const SymFracArgs& A, int a, int b, int lane, float expo,
                                         const float3 (&Sh)[kSymNI], const float3 (&Sl)[kSymNI],
                                         const float (&aS)[kSymNI], const float (&Su)[kSymNI][KC],
                                         float (&sacc)[kSymNI][KC])
{
    constexpr int KP = KPad<KC>::value;
    const float* __restrict__ ub = A.ub;
    const WaveRot rot(lane);
    for (int q = 0; q < kSymFaces / 64; ++q) {
        const int64_t T = (int64_t)b * kSymFaces + q * 64 + lane;
        float4 th = A.fx[T];
        float3 tl = make_float3(0.f, 0.f, 0.f);
        if (LO) {
            const float4 l = A.fl[T];
            tl = make_float3(l.x, l.y, l.z);
        }
        float tu[KC], tacc[KC];
#pragma unroll
        for (int c = 0; c < KC; ++c) {
            tu[c] = ub[T * KP + c];
            tacc[c] = 0.f;
        }
        int ti = (int)T;
#pragma unroll 2
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
                const float g = exp2_fast(expo * log2_fast(r2));
                const float gaT = g * th.w;
                const float gaS = g * aS[r];
#pragma unroll
                for (int c = 0; c < KC; ++c) {
                    const float diff = Su[r][c] - tu[c];
                    sacc[r][c] += gaT * diff;
                    if (!DIAG) tacc[c] += gaS * diff;   // minus row T's sum (negated on the store)
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
#pragma unroll
            for (int c = 0; c < KC; ++c) {
                tu[c] = rot(tu[c]);
                if (!DIAG) tacc[c] = rot(tacc[c]);
            }
            if (DIAG) ti = rot(ti);
        }
        // 64 rotations later every face T is back in its own lane
        if (!DIAG) {
#pragma unroll
            for (int c = 0; c < KC; ++c) A.part[((int64_t)(a - A.a0) * KC + c) * A.ldp + T] = -tacc[c];
        }
    }
}

template <int KC, bool HILO>
__global__ __launch_bounds__(kBlock) void k_frac32_sym(SymFracArgs A, float expo)
{
    constexpr int KP = KPad<KC>::value;
    const int lane = (int)threadIdx.x & 63;
    const int64_t unit = (int64_t)blockIdx.x * (kBlock / 64) + ((int)threadIdx.x >> 6);
    const int nB = A.nB;
    int a, b;
    if (!sym_unit_blocks(unit, nB, A.a0, A.a1, a, b)) return;   // the whole wave leaves
    float3 Sh[kSymNI], Sl[kSymNI];
    float aS[kSymNI], Su[kSymNI][KC], sacc[kSymNI][KC];
#pragma unroll
    for (int r = 0; r < kSymNI; ++r) {
        const int64_t S = (int64_t)a * kSymFaces + r * 64 + lane;
        const float4 x = A.fx[S];
        Sh[r] = make_float3(x.x, x.y, x.z);
        aS[r] = x.w;
        if (HILO) {
            const float4 l = A.fl[S];
            Sl[r] = make_float3(l.x, l.y, l.z);
        } else {
            Sl[r] = make_float3(0.f, 0.f, 0.f);
        }
#pragma unroll
        for (int c = 0; c < KC; ++c) {
            Su[r][c] = A.ub[S * KP + c];
            sacc[r][c] = 0.f;
        }
    }
    if (a == b) {
        sym_unit<KC, HILO, true>(A, a, b, lane, expo, Sh, Sl, aS, Su, sacc);
    } else {
        bool lo = HILO;
        if (HILO) {   // blocks far apart: the high parts suffice (tile_is_far)
            float4 ilo, ihi;
            irange_box(A.tbox, (int64_t)a * kSymFaces, kSymFaces, ilo, ihi);
            lo = false;
            for (int t = 0; t < kSymFaces / kTileJ; ++t)
                lo = lo || !tile_is_far(ilo, ihi, A.tbox, b * (kSymFaces / kTileJ) + t);
        }
        if (lo) sym_unit<KC, HILO, false>(A, a, b, lane, expo, Sh, Sl, aS, Su, sacc);
        else sym_unit<KC, false, false>(A, a, b, lane, expo, Sh, Sl, aS, Su, sacc);
    }
#pragma unroll
    for (int r = 0; r < kSymNI; ++r) {
        const int64_t S = (int64_t)(a - A.a0) * kSymFaces + r * 64 + lane;   // row in the band
#pragma unroll
        for (int c = 0; c < KC; ++c) A.partS[((int64_t)b * KC + c) * A.ldS + S] = sacc[r][c];
    }
}

// ============================================================== symmetric E + dE (FP32)
//
// The same scheme for the energy's differential: an unordered pair (S, T) gives row S's
// eleven sums and row T's.  Seen from T, d, N_T.d and N_S.d change sign exactly, so K and
// K' are shared and the q-derivatives change sign; row T's terms are row S's formulas with
// a_S, N_S in place of a_T, N_T and those signs, bit for bit the terms its own evaluation
// would give.  Row T's first seven sums are kept negated so that every update is a plain
// multiply-add, and put right in the epilogue.

struct GSymArgs {
    const float4* fx = nullptr;
    const float4* fl = nullptr;
    const float4* fn = nullptr;
    const double4* dx = nullptr;
    const double4* dn = nullptr;
    const float4* tbox = nullptr;
    float* part = nullptr;    // row T's sums: [K][kGradOut][ldp]
    float* partS = nullptr;   // row S's sums: [nB][kGradOut][ldS]
    int64_t ldp = 0;
    int64_t ldS = 0;
    int nB = 0;
    int a0 = 0, a1 = 0;       // band of rows
    float rho2 = 0.f;
};

// The seven outputs of face f from its eleven sums (FP64, as in k_grad32), to dst[m * ld].
__device__ __forceinline__ void gsym_store(const GSymArgs& A, float* dst, int64_t ld, int64_t f,
                                           const float (&c)[kGradAcc], double alpha, double beta)
{
    const double aF = A.dx[f].w;
    const double4 N = A.dn[f];
    double a[kGradAcc];
#pragma unroll
    for (int m = 0; m < kGradAcc; ++m) a[m] = (double)c[m];
    dst[0 * ld] = (float)(aF * (alpha * (N.x * a[0] + a[1]) - beta * a[4]));
    dst[1 * ld] = (float)(aF * (alpha * (N.y * a[0] + a[2]) - beta * a[5]));
    dst[2 * ld] = (float)(aF * (alpha * (N.z * a[0] + a[3]) - beta * a[6]));
    dst[3 * ld] = (float)(aF * alpha * a[7]);
    dst[4 * ld] = (float)(aF * alpha * a[8]);
    dst[5 * ld] = (float)(aF * alpha * a[9]);
    dst[6 * ld] = (float)a[10];
}

template <bool LO, bool NEAR, bool DIAG, class Pow>
__device__ __forceinline__ void gsym_unit(const GSymArgs& A, int a, int b, int lane, const Pow& pw, double alpha,
                                          double beta, const float3 (&Sh)[kSymNI], const float3 (&Sl)[kSymNI],
                                          const float3 (&Sn)[kSymNI], const float (&aS)[kSymNI],
                                          float (&c)[kSymNI][kGradAcc])
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
        float ct[kGradAcc];
#pragma unroll
        for (int m = 0; m < kGradAcc; ++m) ct[m] = 0.f;
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
                float r2 = dist2_32(dx, dy, dz);
                if (DIAG) r2 = ((int)((int64_t)a * kSymFaces + r * 64 + lane) == ti) ? 1.0f : r2;
                if (NEAR) r2 = r2 < A.rho2 ? INFINITY : r2;   // summed by the FP64 near field
                const float inv = rcp_fast(r2);
                const float qs = Sn[r].x * dx + Sn[r].y * dy + Sn[r].z * dz;
                const float qt = tn.x * dx + tn.y * dy + tn.z * dz;
                float K, Kqr, Kp, Kpqr;
                pw.KG(qs, r2, inv, K, Kqr);
                pw.KG(qt, r2, inv, Kp, Kpqr);
                const float KK = K + Kp;
                // row S, as k_grad32 forms it
                const float t = th.w * inv;
                const float aq = Kqr * t, ap = Kpqr * t, cc = KK * t;
                c[r][0] += aq;
                c[r][1] += ap * tn.x;
                c[r][2] += ap * tn.y;
                c[r][3] += ap * tn.z;
                c[r][4] += cc * dx;
                c[r][5] += cc * dy;
                c[r][6] += cc * dz;
                c[r][7] += aq * dx;
                c[r][8] += aq * dy;
                c[r][9] += aq * dz;
                c[r][10] += KK * th.w;
                if (!DIAG) {
                    // row T: sums 0..6 negated
                    const float ts = aS[r] * inv;
                    const float bq = Kpqr * ts, bp = Kqr * ts, cs = KK * ts;
                    ct[0] += bq;
                    ct[1] += bp * Sn[r].x;
                    ct[2] += bp * Sn[r].y;
                    ct[3] += bp * Sn[r].z;
                    ct[4] += cs * dx;
                    ct[5] += cs * dy;
                    ct[6] += cs * dz;
                    ct[7] += bq * dx;
                    ct[8] += bq * dy;
                    ct[9] += bq * dz;
                    ct[10] += KK * aS[r];
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
            if (!DIAG) {
#pragma unroll
                for (int m = 0; m < kGradAcc; ++m) ct[m] = rot(ct[m]);
            }
            if (DIAG) ti = rot(ti);
        }
        if (!DIAG) {
#pragma unroll
            for (int m = 0; m < 7; ++m) ct[m] = -ct[m];
            gsym_store(A, A.part + (int64_t)(a - A.a0) * kGradOut * A.ldp + T, A.ldp, T, ct, alpha, beta);
        }
    }
}

template <bool HILO, bool NEAR, class Pow>
__global__ __launch_bounds__(kBlock) void k_grad32_sym(GSymArgs A, double alpha, double beta, Pow pw)
{
    const int lane = (int)threadIdx.x & 63;
    const int64_t unit = (int64_t)blockIdx.x * (kBlock / 64) + ((int)threadIdx.x >> 6);
    const int nB = A.nB;
    int a, b;
    if (!sym_unit_blocks(unit, nB, A.a0, A.a1, a, b)) return;   // the whole wave leaves
    float3 Sh[kSymNI], Sl[kSymNI], Sn[kSymNI];
    float aS[kSymNI], c[kSymNI][kGradAcc];
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
        for (int m = 0; m < kGradAcc; ++m) c[r][m] = 0.f;
    }
    // the block pair's tile tests, as k_grad32 makes them for a tile
    bool near = false, far = HILO;
    if (NEAR || HILO) {
        float4 ilo, ihi;
        irange_box(A.tbox, (int64_t)a * kSymFaces, kSymFaces, ilo, ihi);
        for (int t = 0; t < kSymFaces / kTileJ; ++t) {
            const int jt = b * (kSymFaces / kTileJ) + t;
            if (NEAR) near = near || tile_may_be_near(ilo, ihi, A.tbox, jt, A.rho2);
            if (HILO) far = far && tile_is_far(ilo, ihi, A.tbox, jt);
        }
    }
    if (a == b)
        gsym_unit<HILO, NEAR, true>(A, a, b, lane, pw, alpha, beta, Sh, Sl, Sn, aS, c);
    else if (NEAR && near)
        gsym_unit<HILO, NEAR, false>(A, a, b, lane, pw, alpha, beta, Sh, Sl, Sn, aS, c);
    else if (HILO && far)
        gsym_unit<false, false, false>(A, a, b, lane, pw, alpha, beta, Sh, Sl, Sn, aS, c);
    else
        gsym_unit<HILO, false, false>(A, a, b, lane, pw, alpha, beta, Sh, Sl, Sn, aS, c);
#pragma unroll
    for (int r = 0; r < kSymNI; ++r) {
        const int64_t row = (int64_t)(a - A.a0) * kSymFaces + r * 64 + lane;   // row in the band
        gsym_store(A, A.partS + (int64_t)b * kGradOut * A.ldS + row, A.ldS, (int64_t)a * kSymFaces + r * 64 + lane,
                   c[r], alpha, beta);
    }
}

// ============================================================== symmetric energy (FP32)
//
// The energy alone needs no per-face sums: an unordered pair (S, T) adds
// a_S a_T (K(S,T) + K(T,S)) (a_S a_T K(S,T) on diagonal blocks, where both orders come up),
// so only the faces S of a lane collect, the faces T pass along the wave with their
// positions, areas and normals (7 values a step, 10 with the low parts), and each wave writes
// one FP64 partial for its pair of blocks; the partials are summed in a fixed order.

struct ESymArgs {
    const float4* fx = nullptr;
    const float4* fl = nullptr;
    const float4* fn = nullptr;
    const float4* tbox = nullptr;
    double* upart = nullptr;   // one partial per pair of blocks
    int64_t nF = 0;
    int nB = 0;
    float rho2 = 0.f;
};

template <bool LO, bool NEAR, bool DIAG, class Pow>
__device__ __forceinline__ void esym_unit(const ESymArgs& A, int a, int b, int lane, const Pow& pw,
                                          const float3 (&Sh)[kSymNI], const float3 (&Sl)[kSymNI],
                                          const float3 (&Sn)[kSymNI], double (&acc)[kSymNI])
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
        int ti = (int)T;
        float c[kSymNI];
#pragma unroll
        for (int r = 0; r < kSymNI; ++r) c[r] = 0.f;
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
                float r2 = dist2_32(dx, dy, dz);
                if (DIAG) r2 = ((int)((int64_t)a * kSymFaces + r * 64 + lane) == ti) ? 1.0f : r2;
                if (NEAR) r2 = r2 < A.rho2 ? INFINITY : r2;   // summed by the FP64 near field
                const float inv = rcp_fast(r2);
                const float qs = Sn[r].x * dx + Sn[r].y * dy + Sn[r].z * dz;
                float K = pw.K(qs, r2, inv);
                if (!DIAG) {
                    const float qt = tn.x * dx + tn.y * dy + tn.z * dz;
                    K += pw.K(qt, r2, inv);
                }
                c[r] += K * th.w;
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
            if (!DIAG) {
                tn.x = rot(tn.x);
                tn.y = rot(tn.y);
                tn.z = rot(tn.z);
            }
            if (DIAG) ti = rot(ti);
        }
#pragma unroll
        for (int r = 0; r < kSymNI; ++r) acc[r] += (double)c[r];
    }
}

template <bool HILO, bool NEAR, class Pow>
__global__ __launch_bounds__(kBlock) void k_energy32_sym(ESymArgs A, Pow pw)
{
    const int lane = (int)threadIdx.x & 63;
    const int64_t unit = (int64_t)blockIdx.x * (kBlock / 64) + ((int)threadIdx.x >> 6);
    const int nB = A.nB;
    int a, b;
    if (!sym_unit_blocks(unit, nB, 0, nB, a, b)) return;   // the whole wave leaves
    float3 Sh[kSymNI], Sl[kSymNI], Sn[kSymNI];
    float aS[kSymNI];
    double acc[kSymNI];
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
        acc[r] = 0.0;
    }
    bool near = false, far = HILO;
    if (NEAR || HILO) {
        float4 ilo, ihi;
        irange_box(A.tbox, (int64_t)a * kSymFaces, kSymFaces, ilo, ihi);
        for (int t = 0; t < kSymFaces / kTileJ; ++t) {
            const int jt = b * (kSymFaces / kTileJ) + t;
            if (NEAR) near = near || tile_may_be_near(ilo, ihi, A.tbox, jt, A.rho2);
            if (HILO) far = far && tile_is_far(ilo, ihi, A.tbox, jt);
        }
    }
    if (a == b)
        esym_unit<HILO, NEAR, true>(A, a, b, lane, pw, Sh, Sl, Sn, acc);
    else if (NEAR && near)
        esym_unit<HILO, NEAR, false>(A, a, b, lane, pw, Sh, Sl, Sn, acc);
    else if (HILO && far)
        esym_unit<false, false, false>(A, a, b, lane, pw, Sh, Sl, Sn, acc);
    else
        esym_unit<HILO, false, false>(A, a, b, lane, pw, Sh, Sl, Sn, acc);
    // the lane's faces S (padding faces, which can meet each other at distance 0, left out),
    // then the wave's sum by an xor butterfly: every lane adds the same two values in the
    // same order, so all lanes hold the same bits
    double e = 0.0;
#pragma unroll
    for (int r = 0; r < kSymNI; ++r)
        if ((int64_t)a * kSymFaces + r * 64 + lane < A.nF) e += (double)aS[r] * acc[r];
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) e += __shfl_xor(e, m, 64);
    if (lane == 0) A.upart[unit] = e;
}

// out[i] = a_i near[i] (the near field's share of the energy per face), i < n.
__global__ void k_area_times(const double4* __restrict__ dx, const double* __restrict__ near, int64_t n,
                             double* __restrict__ out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = dx[i].w * near[i];
}

// The band [a0, a1) of rows, for faces i >= a0 kSymFaces (the others get nothing from it):
// out[c][i] (0 before the first band) plus, in FP64 and in slice order, row T's slices
// a in [a0, min(a1, block of i)), then, for faces of the band, row S's slices b >= block of
// i and extra[c][i] (the FP64 near field, when given).  Over all bands that is the slice
// order a = 0 .. nB - 1 of a single launch.
__global__ void k_reduce_sym_band(const float* __restrict__ partT, const float* __restrict__ partS, int nB, int a0,
                                  int a1, int kc, int64_t ldp, int64_t ldS, int64_t n, const double* __restrict__ extra,
                                  double* __restrict__ out, int64_t out_stride)
{
    const int64_t i0 = (int64_t)a0 * kSymFaces, m = n - i0;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (m <= 0 || t >= m * kc) return;
    const int c = (int)(t / m);
    const int64_t i = i0 + (t - (int64_t)c * m);
    const int blk = (int)(i / kSymFaces);
    double* o = out + (int64_t)c * out_stride + i;
    double s = a0 == 0 ? 0.0 : *o;
    // s += p[0], p[stride], ... in that order; the loads of 16 slices are issued together
    auto add_slices = [&s](const float* __restrict__ p, int64_t stride, int cnt) {
        constexpr int U = 16;
        int j = 0;
        for (; j + U <= cnt; j += U) {
            float v[U];
#pragma unroll
            for (int u = 0; u < U; ++u) v[u] = p[(int64_t)(j + u) * stride];
#pragma unroll
            for (int u = 0; u < U; ++u) s += (double)v[u];
        }
        for (; j < cnt; ++j) s += (double)p[(int64_t)j * stride];
    };
    const int ta = min(a1, blk);
    if (ta > a0) add_slices(partT + (int64_t)c * ldp + i, (int64_t)kc * ldp, ta - a0);
    if (blk < a1) {
        add_slices(partS + ((int64_t)blk * kc + c) * ldS + (i - i0), (int64_t)kc * ldS, nB - blk);
        if (extra) s += extra[(int64_t)c * out_stride + i];
    }
    *o = s;
}

// ============================================================== FP64 variants
//
// Same structure with double pair terms and no per-tile FP32 stage.

__device__ __forceinline__ void load_tile64(const double4* __restrict__ dxa,
                                            const double4* __restrict__ dn, double4* s_x,
                                            double4* s_n, int64_t j0, bool with_n)
{
    for (int e = threadIdx.x; e < kTileJ; e += kBlock) {
        s_x[e] = dxa[j0 + e];
        if (with_n) s_n[e] = dn[j0 + e];
    }
}

template <bool DIAG, class Pow>
__device__ __forceinline__ void energy_tile64(const double4* s_x, int64_t j0, double3 S, double3 N,
                                              int64_t Si, const Pow& pw, double& c)
{
#pragma unroll 2
    for (int jj = 0; jj < kTileJ; ++jj) {
        const double4 t = s_x[jj];
        double dx = S.x - t.x, dy = S.y - t.y, dz = S.z - t.z;
        double r2 = dx * dx + dy * dy + dz * dz;
        if (DIAG) r2 = (Si == j0 + jj) ? 1.0 : r2;
        const double inv = rcp_fast(r2);
        const double q = N.x * dx + N.y * dy + N.z * dz;
        c += pw.K(q, r2, inv) * t.w;
    }
}

template <class Pow>
__global__ __launch_bounds__(kBlock) void k_energy64(PairBatch jb, Pow pw)
{
    const PairJob J = pick_job(jb);
    const int bi = ((int)blockIdx.x - J.block0) % J.n_itiles;
    const int bs = ((int)blockIdx.x - J.block0) / J.n_itiles;
    const int tiles_per_split = J.tiles_per_split, ntiles_j = J.ntiles_j;
    double* __restrict__ part = J.part;
    const int64_t irows = J.irows;
    const double4* __restrict__ dxa = J.dx;
    const double4* __restrict__ dn = J.dn;
    __shared__ double4 s_x[kTileJ];
    const int64_t ibase = (int64_t)bi * kBlock;
    const int jt0 = bs * tiles_per_split;
    const int jt1 = min(jt0 + tiles_per_split, ntiles_j);
    const int64_t Si = ibase + threadIdx.x;
    const double4 x = dxa[Si], n = dn[Si];
    const double3 S = make_double3(x.x, x.y, x.z), N = make_double3(n.x, n.y, n.z);
    double acc = 0.0;
    for (int jt = jt0; jt < jt1; ++jt) {
        const int64_t j0 = (int64_t)jt * kTileJ;
        __syncthreads();
        load_tile64(dxa, dn, s_x, nullptr, j0, false);
        __syncthreads();
        if (tile_hits_diag(j0, ibase, kBlock)) energy_tile64<true>(s_x, j0, S, N, Si, pw, acc);
        else energy_tile64<false>(s_x, j0, S, N, Si, pw, acc);
    }
    part[(int64_t)bs * irows + Si] = acc;
}

template <bool DIAG, class Pow>
__device__ __forceinline__ void grad_tile64(const double4* s_x, const double4* s_n, int64_t j0,
                                            double3 S, double3 N, int64_t Si, const Pow& pw,
                                            double (&c)[kGradAcc])
{
#pragma unroll 2
    for (int jj = 0; jj < kTileJ; ++jj) {
        const double4 tx = s_x[jj];
        const double4 tn = s_n[jj];
        const double aT = tx.w;
        double dx = S.x - tx.x, dy = S.y - tx.y, dz = S.z - tx.z;
        double r2 = dx * dx + dy * dy + dz * dz;
        if (DIAG) r2 = (Si == j0 + jj) ? 1.0 : r2;
        const double inv = rcp_fast(r2);
        const double q = N.x * dx + N.y * dy + N.z * dz;
        const double qp = tn.x * dx + tn.y * dy + tn.z * dz;
        double K, Kqr, Kp, Kpqr;
        pw.KG(q, r2, inv, K, Kqr);
        pw.KG(qp, r2, inv, Kp, Kpqr);
        const double t = aT * inv;
        const double aq = Kqr * t;
        const double ap = Kpqr * t;
        const double KK = K + Kp;
        const double cc = KK * t;
        c[0] += aq;
        c[1] += ap * tn.x;
        c[2] += ap * tn.y;
        c[3] += ap * tn.z;
        c[4] += cc * dx;
        c[5] += cc * dy;
        c[6] += cc * dz;
        c[7] += aq * dx;
        c[8] += aq * dy;
        c[9] += aq * dz;
        c[10] += KK * aT;
    }
}

template <class Pow>
__global__ __launch_bounds__(kBlock) void k_grad64(PairBatch jb, double alpha, double beta, Pow pw)
{
    const PairJob J = pick_job(jb);
    const int bi = ((int)blockIdx.x - J.block0) % J.n_itiles;
    const int bs = ((int)blockIdx.x - J.block0) / J.n_itiles;
    const int tiles_per_split = J.tiles_per_split, ntiles_j = J.ntiles_j;
    double* __restrict__ part = J.part;
    const int64_t irows = J.irows;
    const double4* __restrict__ dxa = J.dx;
    const double4* __restrict__ dn = J.dn;
    __shared__ double4 s_x[kTileJ], s_n[kTileJ];
    const int64_t ibase = (int64_t)bi * kBlock;
    const int jt0 = bs * tiles_per_split;
    const int jt1 = min(jt0 + tiles_per_split, ntiles_j);
    const int64_t Si = ibase + threadIdx.x;
    const double4 x = dxa[Si], n = dn[Si];
    const double3 S = make_double3(x.x, x.y, x.z), N = make_double3(n.x, n.y, n.z);
    double a[kGradAcc];
#pragma unroll
    for (int m = 0; m < kGradAcc; ++m) a[m] = 0.0;
    for (int jt = jt0; jt < jt1; ++jt) {
        const int64_t j0 = (int64_t)jt * kTileJ;
        __syncthreads();
        load_tile64(dxa, dn, s_x, s_n, j0, true);
        __syncthreads();
        if (tile_hits_diag(j0, ibase, kBlock)) grad_tile64<true>(s_x, s_n, j0, S, N, Si, pw, a);
        else grad_tile64<false>(s_x, s_n, j0, S, N, Si, pw, a);
    }
    const double aS = x.w;
    double out[kGradOut];
    out[0] = aS * (alpha * (N.x * a[0] + a[1]) - beta * a[4]);
    out[1] = aS * (alpha * (N.y * a[0] + a[2]) - beta * a[5]);
    out[2] = aS * (alpha * (N.z * a[0] + a[3]) - beta * a[6]);
    out[3] = aS * alpha * a[7];
    out[4] = aS * alpha * a[8];
    out[5] = aS * alpha * a[9];
    out[6] = a[10];
    double* dst = part + (int64_t)bs * kGradOut * irows + Si;
#pragma unroll
    for (int m = 0; m < kGradOut; ++m) dst[m * irows] = out[m];
}

template <int KC>
__global__ __launch_bounds__(kBlock) void k_frac64(PairBatch jb, double expo)
{
    const PairJob J = pick_job(jb);
    const int bi = ((int)blockIdx.x - J.block0) % J.n_itiles;
    const int bs = ((int)blockIdx.x - J.block0) / J.n_itiles;
    const int tiles_per_split = J.tiles_per_split, ntiles_j = J.ntiles_j;
    double* __restrict__ part = J.part;
    const int64_t irows = J.irows;
    const double4* __restrict__ dxa = J.dx;
    const double* __restrict__ ub = static_cast<const double*>(J.ub);
    constexpr int KP = KPad<KC>::value;
    __shared__ double4 s_x[kTileJ];
    __shared__ double s_u[kTileJ * KP];
    const int64_t ibase = (int64_t)bi * kBlock;
    const int jt0 = bs * tiles_per_split;
    const int jt1 = min(jt0 + tiles_per_split, ntiles_j);
    const int64_t Si = ibase + threadIdx.x;
    const double4 x = dxa[Si];
    double Su[KC], acc[KC];
#pragma unroll
    for (int cc = 0; cc < KC; ++cc) {
        Su[cc] = ub[Si * KP + cc];
        acc[cc] = 0.0;
    }
    for (int jt = jt0; jt < jt1; ++jt) {
        const int64_t j0 = (int64_t)jt * kTileJ;
        __syncthreads();
        for (int e = threadIdx.x; e < kTileJ; e += kBlock) s_x[e] = dxa[j0 + e];
        for (int e = threadIdx.x; e < kTileJ * KP; e += kBlock) s_u[e] = ub[j0 * KP + e];
        __syncthreads();
        const bool diag = tile_hits_diag(j0, ibase, kBlock);
        for (int jj = 0; jj < kTileJ; ++jj) {
            const double4 t = s_x[jj];
            double dx = x.x - t.x, dy = x.y - t.y, dz = x.z - t.z;
            double r2 = dx * dx + dy * dy + dz * dz;
            if (diag && Si == j0 + jj) continue;
            const double w = pow(r2, expo) * t.w;
#pragma unroll
            for (int cc = 0; cc < KC; ++cc) acc[cc] += w * (Su[cc] - s_u[jj * KP + cc]);
        }
    }
#pragma unroll
    for (int cc = 0; cc < KC; ++cc) part[((int64_t)bs * KC + cc) * irows + Si] = acc[cc];
}

// ============================================================== FP64 near field
//
// A pair (S, T), T != S, is near when its FP32 hi+lo squared distance, formed exactly as
// in the FP32 kernels, is below rho2; near pairs are summed in FP64 with the same
// accumulators and epilogue as the all-pairs kernels (row ownership: S collects the (S,T)
// and (T,S) terms).  Only j-tiles whose box lies within the near radius of the i-range box
// are visited.

template <bool GEN>
__device__ __forceinline__ void kg64(double q, double r2, double inv, double alpha, double beta, double& K,
                                     double& Kqr)
{
    if (!GEN) {
        const double u = q * inv, u2 = u * u, u4 = u2 * u2;
        K = u4 * u2;
        Kqr = u4 * u;
    } else if (q == 0.0) {
        K = 0.0;
        Kqr = 0.0;
    } else {
        Kqr = copysign(pow(fabs(q), alpha - 1.0) * pow(r2, 1.0 - 0.5 * beta), q);
        K = Kqr * q * inv;
    }
}

constexpr int kNearBlock = 128;    // threads per near-field workgroup
constexpr int kNearLanes = 8;      // lanes that share the candidates of one face S
constexpr int kNearFaces = kNearBlock / kNearLanes;   // faces S per workgroup
static_assert(kNearBlock % kNearLanes == 0 && 64 % kNearLanes == 0, "a face's lanes lie in one wave");

// Cell of an FP32 barycenter: floor((x - lo) inv_cs) per axis, clamped to [0, g).
__device__ __forceinline__ int near_cell_axis(float x, float lo, float inv_cs, int g)
{
    const int c = (int)floorf((x - lo) * inv_cs);
    return c < 0 ? 0 : (c >= g ? g - 1 : c);
}

// Sum over the kNearLanes lanes of a face by an xor butterfly: every lane ends with the
// same bits (for four lanes (v0 + v1) + (v2 + v3)), whatever the order the lanes ran in.
__device__ __forceinline__ double near_lane_sum(double v)
{
#pragma unroll
    for (int o = 1; o < kNearLanes; o <<= 1) v += __shfl_xor(v, o, kNearLanes);
    return v;
}

// A workgroup takes kNearFaces consecutive faces of the cell order (faces of a wave share
// cells, so their candidate loops run nearly in step), kNearLanes lanes per face.  Face S
// visits the 27 cells around its own in a fixed order and, in each, the faces in cell
// order; lane l of S takes every kNearLanes-th of them from the l-th on.  For every
// candidate T the lane forms the FP32 hi+lo squared distance exactly as the FP32 kernels
// do, and evaluates the pair in FP64 when that distance is below rho2.  Each lane's sums
// have a fixed order, and so has their combination (near_lane_sum).
template <bool GEN, bool GRAD>
__global__ __launch_bounds__(kNearBlock) void k_near64(PairBatch jb, double alpha, double beta)
{
    const PairJob J = pick_job(jb);
    const NearGridParams G = *J.ngp;
    const int lane = (int)threadIdx.x % kNearLanes;
    const int i = ((int)blockIdx.x - J.block0) * kNearFaces + (int)threadIdx.x / kNearLanes;
    if (i >= G.n) return;   // all lanes of a face leave together
    const int S = J.nord[i];
    const float4 sh = J.nfx[i], sl = J.nfl[i];
    const double4 X = J.dx[S], Nn = J.dn[S];
    const int cx = near_cell_axis(sh.x, G.lo[0], G.inv_cs, G.g);
    const int cy = near_cell_axis(sh.y, G.lo[1], G.inv_cs, G.g);
    const int cz = near_cell_axis(sh.z, G.lo[2], G.inv_cs, G.g);
    double c[11];
#pragma unroll
    for (int m = 0; m < 11; ++m) c[m] = 0.0;
    double e = 0.0;
    for (int z = max(cz - 1, 0); z <= min(cz + 1, G.g - 1); ++z)
        for (int y = max(cy - 1, 0); y <= min(cy + 1, G.g - 1); ++y)
            for (int x = max(cx - 1, 0); x <= min(cx + 1, G.g - 1); ++x) {
                const int2 be = J.ncell[((int64_t)z * G.g + y) * G.g + x];
                for (int j = be.x + lane; j < be.y; j += kNearLanes) {
                    const float4 th = J.nfx[j], tl = J.nfl[j];
                    const float fdx = (sh.x - th.x) + (sl.x - tl.x);
                    const float fdy = (sh.y - th.y) + (sl.y - tl.y);
                    const float fdz = (sh.z - th.z) + (sl.z - tl.z);
                    if (!(dist2_32(fdx, fdy, fdz) < J.rho2) || j == i) continue;
                    const int T = J.nord[j];
                    const double4 Y = J.dx[T], Nt = J.dn[T];
                    const double dx = X.x - Y.x, dy = X.y - Y.y, dz = X.z - Y.z;
                    const double r2 = dx * dx + dy * dy + dz * dz;
                    const double inv = 1.0 / r2;
                    const double q = Nn.x * dx + Nn.y * dy + Nn.z * dz;
                    double K, Kqr;
                    kg64<GEN>(q, r2, inv, alpha, beta, K, Kqr);
                    if (!GRAD) {
                        e += K * Y.w;
                        continue;
                    }
                    const double qp = Nt.x * dx + Nt.y * dy + Nt.z * dz;
                    double Kp, Kpqr;
                    kg64<GEN>(qp, r2, inv, alpha, beta, Kp, Kpqr);
                    const double tt = Y.w * inv;
                    const double aq = Kqr * tt, ap = Kpqr * tt, KK = K + Kp, cc = KK * tt;
                    c[0] += aq;
                    c[1] += ap * Nt.x;
                    c[2] += ap * Nt.y;
                    c[3] += ap * Nt.z;
                    c[4] += cc * dx;
                    c[5] += cc * dy;
                    c[6] += cc * dz;
                    c[7] += aq * dx;
                    c[8] += aq * dy;
                    c[9] += aq * dz;
                    c[10] += KK * Y.w;
                }
            }
    if (!GRAD) {
        e = near_lane_sum(e);
        if (lane == 0) J.part[S] = e;
        return;
    }
#pragma unroll
    for (int m = 0; m < 11; ++m) c[m] = near_lane_sum(c[m]);
    if (lane != 0) return;
    const double aS = X.w;
    double o[7];
    o[0] = aS * (alpha * (Nn.x * c[0] + c[1]) - beta * c[4]);
    o[1] = aS * (alpha * (Nn.y * c[0] + c[2]) - beta * c[5]);
    o[2] = aS * (alpha * (Nn.z * c[0] + c[3]) - beta * c[6]);
    o[3] = aS * alpha * c[7];
    o[4] = aS * alpha * c[8];
    o[5] = aS * alpha * c[9];
    o[6] = c[10];
#pragma unroll
    for (int m = 0; m < 7; ++m) J.part[m * J.irows + S] = o[m];
}

// ------------------------------------------------------------------ near-field grid build

// Grid parameters from the tile boxes (one workgroup): the cube around the box of all
// FP32 barycenters, g = floor(extent / (1.01 near radius)) cells per axis, 1 <= g <= gmax.
__global__ __launch_bounds__(256) void k_near_grid_params(const float4* __restrict__ tbox, int ntiles, int64_t nF,
                                                          float rho2, int gmax, NearGridParams* __restrict__ out)
{
    __shared__ float sh[6][256];
    float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int t = threadIdx.x; t < ntiles; t += 256) {
        const float4 a = tbox[2 * t], b = tbox[2 * t + 1];
        lo[0] = fminf(lo[0], a.x); lo[1] = fminf(lo[1], a.y); lo[2] = fminf(lo[2], a.z);
        hi[0] = fmaxf(hi[0], b.x); hi[1] = fmaxf(hi[1], b.y); hi[2] = fmaxf(hi[2], b.z);
    }
    for (int m = 0; m < 3; ++m) {
        sh[m][threadIdx.x] = lo[m];
        sh[3 + m][threadIdx.x] = hi[m];
    }
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int m = 0; m < 3; ++m) {
                sh[m][threadIdx.x] = fminf(sh[m][threadIdx.x], sh[m][threadIdx.x + w]);
                sh[3 + m][threadIdx.x] = fmaxf(sh[3 + m][threadIdx.x], sh[3 + m][threadIdx.x + w]);
            }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        NearGridParams P;
        float ext = 0.f;
        for (int m = 0; m < 3; ++m) {
            P.lo[m] = sh[m][0];
            ext = fmaxf(ext, sh[3 + m][0] - sh[m][0]);
        }
        const float r = 1.01f * sqrtf(rho2);
        int g = (r > 0.f && ext > 0.f) ? (int)fminf((float)gmax, floorf(ext / r)) : 1;
        g = g < 1 ? 1 : g;
        P.g = g;
        P.inv_cs = ext > 0.f ? (float)g / ext : 0.f;
        P.n = (int)nF;
        *out = P;
    }
}

__global__ void k_near_grid_keys(const float4* __restrict__ fx, int64_t nF, const NearGridParams* __restrict__ prm,
                                 uint32_t* __restrict__ key, int32_t* __restrict__ val)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= nF) return;
    const NearGridParams G = *prm;
    const float4 p = fx[s];
    const int cx = near_cell_axis(p.x, G.lo[0], G.inv_cs, G.g);
    const int cy = near_cell_axis(p.y, G.lo[1], G.inv_cs, G.g);
    const int cz = near_cell_axis(p.z, G.lo[2], G.inv_cs, G.g);
    key[s] = (uint32_t)(((int64_t)cz * G.g + cy) * G.g + cx);
    val[s] = (int32_t)s;
}

__global__ void k_near_grid_clear(int2* __restrict__ cell, int64_t n)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) cell[t] = make_int2(0, 0);
}

// Cell ranges and the face records in cell order.
__global__ void k_near_grid_mark(const uint32_t* __restrict__ key, const int32_t* __restrict__ val, int64_t nF,
                                 const float4* __restrict__ fx, const float4* __restrict__ fl, int2* __restrict__ cell,
                                 float4* __restrict__ sfx, float4* __restrict__ sfl)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nF) return;
    const uint32_t k = key[i];
    if (i == 0 || key[i - 1] != k) cell[k].x = (int)i;
    if (i == nF - 1 || key[i + 1] != k) cell[k].y = (int)(i + 1);
    const int32_t s = val[i];
    sfx[i] = fx[s];
    sfl[i] = fl[s];
}

// ============================================================== split reduction

__global__ void k_reduce_splits(const double* __restrict__ part, int n_split, int nacc,
                                int64_t irows, int64_t n, double* __restrict__ out,
                                int64_t out_stride)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * nacc) return;
    const int acc = (int)(t / n);
    const int64_t i = t - (int64_t)acc * n;
    double s = 0.0;
    for (int sp = 0; sp < n_split; ++sp) s += part[((int64_t)sp * nacc + acc) * irows + i];
    out[(int64_t)acc * out_stride + i] = s;
}

hipError_t launch_reduce_splits(const double* part, int n_split, int nacc, int64_t irows,
                                int64_t n, double* out, int64_t out_stride, hipStream_t s)
{
    const int64_t total = n * nacc;
    if (total == 0) return hipSuccess;
    hipLaunchKernelGGL(k_reduce_splits, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s,
                       part, n_split, nacc, irows, n, out, out_stride);
    return hipGetLastError();
}

// ============================================================== planning and launch

int64_t face_capacity(int64_t nF, int ni_max)
{
    const int64_t g = (int64_t)kBlock * ni_max;
    int64_t cap = (nF + g - 1) / g * g;
    return std::max<int64_t>(cap, kTileJ);
}

PairPlan plan_pairs(int64_t nF, int64_t cap, int ni, int occupancy_per_cu)
{
    PairPlan pl;
    pl.ni = ni;
    const int64_t ispan = (int64_t)kBlock * ni;
    pl.n_itiles = (int)((nF + ispan - 1) / ispan);
    pl.irows = (int64_t)pl.n_itiles * ispan;
    pl.ntiles_j = (int)((nF + kTileJ - 1) / kTileJ);
    (void)cap;
    const int64_t slots = std::max<int64_t>(1, (int64_t)device_info().num_cu * std::max(1, occupancy_per_cu));
    double best = 1e300;
    int best_tps = pl.ntiles_j;
    for (int tps = 1; tps <= pl.ntiles_j; ++tps) {
        const int64_t ns = (pl.ntiles_j + tps - 1) / tps;
        if (tps > 1 && (pl.ntiles_j + tps - 2) / (tps - 1) == ns) continue;  // same split count
        const int64_t wg = (int64_t)pl.n_itiles * ns;
        const int64_t waves = (wg + slots - 1) / slots;
        // makespan in tiles, plus a small charge per split for the partial sums
        const double cost = (double)waves * tps + 0.05 * (double)ns;
        if (cost < best) {
            best = cost;
            best_tps = tps;
        }
    }
    pl.tiles_per_split = best_tps;
    pl.n_split = (pl.ntiles_j + best_tps - 1) / best_tps;
    return pl;
}

namespace {

// Occupancy (workgroups per CU) of a kernel, queried once per function.
int occupancy_of(const void* fn)
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

bool is_p6(double alpha, double beta) { return alpha == 6.0 && beta == 12.0; }

PowGen make_gen(double alpha, double beta)
{
    PowGen g;
    g.am1 = (float)(alpha - 1.0);
    g.gam = (float)(alpha - 0.5 * beta);
    g.am1d = alpha - 1.0;
    g.hbd = beta * 0.5;
    return g;
}

constexpr int kNiEnergy32 = 4, kNiGrad32 = 2, kNiFrac32 = 2;

const void* energy_fn(int precision, bool p6)
{
    if (precision == TP_PREC_FP64)
        return p6 ? (const void*)k_energy64<PowP6> : (const void*)k_energy64<PowGen>;
    if (precision == TP_PREC_FP32_NEAR64)
        return p6 ? (const void*)k_energy32<kNiEnergy32, true, true, PowP6>
                  : (const void*)k_energy32<kNiEnergy32, true, true, PowGen>;
    if (precision == TP_PREC_FP32_ACC32)
        return p6 ? (const void*)k_energy32<kNiEnergy32, false, false, PowP6, kAcc32>
                  : (const void*)k_energy32<kNiEnergy32, false, false, PowGen, kAcc32>;
    if (precision == TP_PREC_FP32_KAHAN)
        return p6 ? (const void*)k_energy32<kNiEnergy32, false, false, PowP6, kAccKahan>
                  : (const void*)k_energy32<kNiEnergy32, false, false, PowGen, kAccKahan>;
    const bool hilo = precision == TP_PREC_FP32_HILO;
    if (p6) return hilo ? (const void*)k_energy32<kNiEnergy32, true, false, PowP6>
                        : (const void*)k_energy32<kNiEnergy32, false, false, PowP6>;
    return hilo ? (const void*)k_energy32<kNiEnergy32, true, false, PowGen>
                : (const void*)k_energy32<kNiEnergy32, false, false, PowGen>;
}

const void* grad_fn(int precision, bool p6)
{
    if (precision == TP_PREC_FP64)
        return p6 ? (const void*)k_grad64<PowP6> : (const void*)k_grad64<PowGen>;
    if (precision == TP_PREC_FP32_NEAR64)
        return p6 ? (const void*)k_grad32<kNiGrad32, true, true, PowP6>
                  : (const void*)k_grad32<kNiGrad32, true, true, PowGen>;
    if (precision == TP_PREC_FP32_ACC32)
        return p6 ? (const void*)k_grad32<kNiGrad32, false, false, PowP6, kAcc32>
                  : (const void*)k_grad32<kNiGrad32, false, false, PowGen, kAcc32>;
    if (precision == TP_PREC_FP32_KAHAN)
        return p6 ? (const void*)k_grad32<kNiGrad32, false, false, PowP6, kAccKahan>
                  : (const void*)k_grad32<kNiGrad32, false, false, PowGen, kAccKahan>;
    const bool hilo = precision == TP_PREC_FP32_HILO;
    if (p6) return hilo ? (const void*)k_grad32<kNiGrad32, true, false, PowP6>
                        : (const void*)k_grad32<kNiGrad32, false, false, PowP6>;
    return hilo ? (const void*)k_grad32<kNiGrad32, true, false, PowGen>
                : (const void*)k_grad32<kNiGrad32, false, false, PowGen>;
}

template <int KC>
const void* frac_fn_k(int precision)
{
    if (precision == TP_PREC_FP64) return (const void*)k_frac64<KC>;
    if (precision == TP_PREC_FP32_HILO || precision == TP_PREC_FP32_NEAR64)
        return (const void*)k_frac32<kNiFrac32, KC, true>;
    return (const void*)k_frac32<kNiFrac32, KC, false>;
}

const void* frac_fn(int precision, int k)
{
    switch (k) {
    case 1: return frac_fn_k<1>(precision);
    case 2: return frac_fn_k<2>(precision);
    case 3: return frac_fn_k<3>(precision);
    case 4: return frac_fn_k<4>(precision);
    case 5: return frac_fn_k<5>(precision);
    case 6: return frac_fn_k<6>(precision);
    case 7: return frac_fn_k<7>(precision);
    case 8: return frac_fn_k<8>(precision);
    case 9: return frac_fn_k<9>(precision);
    default: return nullptr;
    }
}

int ni_of(int kind, int precision)
{
    if (precision == TP_PREC_FP64) return 1;
    return kind == kKindEnergy ? kNiEnergy32 : (kind == kKindGrad ? kNiGrad32 : kNiFrac32);
}

}  // namespace

PairPlan plan_for(int kind, int precision, int k, int64_t nF, int64_t cap)
{
    const void* fn = kind == kKindEnergy ? energy_fn(precision, true)
                   : kind == kKindGrad   ? grad_fn(precision, true)
                                         : frac_fn(precision, std::max(1, std::min(k, kMaxGroupCols)));
    return plan_pairs(nF, cap, ni_of(kind, precision), occupancy_of(fn));
}

PairJob make_pair_job(const FaceData& fd, const PairPlan& pl, double* part, const void* ub)
{
    PairJob J;
    J.fx = fd.fx; J.fl = fd.fl; J.fn = fd.fn; J.dx = fd.dx; J.dn = fd.dn; J.tbox = fd.tbox;
    J.ub = ub;
    J.part = part;
    J.irows = pl.irows;
    J.n_itiles = pl.n_itiles;
    J.tiles_per_split = pl.tiles_per_split;
    J.ntiles_j = pl.ntiles_j;
    J.block0 = 0;
    return J;
}

namespace {

int job_blocks(const PairJob& J)
{
    const int ns = (J.ntiles_j + J.tiles_per_split - 1) / J.tiles_per_split;
    return J.n_itiles * ns;
}

// Cut the job list into launches of at most kMaxPairJobs jobs, longest workgroups first
// (the order changes no result), and call launch(batch, grid) for each.
template <class F>
hipError_t for_each_batch(const PairJob* jobs, int njobs, F&& launch)
{
    if (njobs < 1) return hipSuccess;
    std::vector<int> order(njobs);
    for (int m = 0; m < njobs; ++m) order[m] = m;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        return jobs[a].tiles_per_split > jobs[b].tiles_per_split;
    });
    for (int m0 = 0; m0 < njobs; m0 += kMaxPairJobs) {
        PairBatch jb;
        jb.n = std::min(kMaxPairJobs, njobs - m0);
        int64_t blocks = 0;
        for (int q = 0; q < kMaxPairJobs; ++q) {
            if (q < jb.n) {
                jb.j[q] = jobs[order[m0 + q]];
                jb.j[q].block0 = (int)blocks;
                blocks += job_blocks(jb.j[q]);
            } else {
                jb.j[q] = jb.j[0];
                jb.j[q].block0 = INT32_MAX;
            }
        }
        if (blocks <= 0) continue;
        if (blocks > (int64_t)INT32_MAX) return hipErrorInvalidValue;
        launch(jb, dim3((unsigned)blocks));
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace

hipError_t launch_pairs_energy(const PairJob* jobs, int njobs, int precision, double alpha,
                               double beta, hipStream_t s)
{
    const dim3 block(kBlock);
    const bool p6 = is_p6(alpha, beta);
    const PowGen g = make_gen(alpha, beta);
    return for_each_batch(jobs, njobs, [&](const PairBatch& jb, dim3 grid) {
        if (precision == TP_PREC_FP64) {
            if (p6) hipLaunchKernelGGL(k_energy64<PowP6>, grid, block, 0, s, jb, PowP6{});
            else hipLaunchKernelGGL(k_energy64<PowGen>, grid, block, 0, s, jb, g);
        } else if (precision == TP_PREC_FP32_NEAR64) {
            if (p6) hipLaunchKernelGGL((k_energy32<kNiEnergy32, true, true, PowP6>), grid, block, 0, s, jb, PowP6{});
            else hipLaunchKernelGGL((k_energy32<kNiEnergy32, true, true, PowGen>), grid, block, 0, s, jb, g);
        } else if (precision == TP_PREC_FP32_ACC32) {
            if (p6) hipLaunchKernelGGL((k_energy32<kNiEnergy32, false, false, PowP6, kAcc32>), grid, block, 0, s, jb, PowP6{});
            else hipLaunchKernelGGL((k_energy32<kNiEnergy32, false, false, PowGen, kAcc32>), grid, block, 0, s, jb, g);
        } else if (precision == TP_PREC_FP32_KAHAN) {
            if (p6) hipLaunchKernelGGL((k_energy32<kNiEnergy32, false, false, PowP6, kAccKahan>), grid, block, 0, s, jb, PowP6{});
            else hipLaunchKernelGGL((k_energy32<kNiEnergy32, false, false, PowGen, kAccKahan>), grid, block, 0, s, jb, g);
        } else if (precision == TP_PREC_FP32_HILO) {
            if (p6) hipLaunchKernelGGL((k_energy32<kNiEnergy32, true, false, PowP6>), grid, block, 0, s, jb, PowP6{});
            else hipLaunchKernelGGL((k_energy32<kNiEnergy32, true, false, PowGen>), grid, block, 0, s, jb, g);
        } else {
            if (p6) hipLaunchKernelGGL((k_energy32<kNiEnergy32, false, false, PowP6>), grid, block, 0, s, jb, PowP6{});
            else hipLaunchKernelGGL((k_energy32<kNiEnergy32, false, false, PowGen>), grid, block, 0, s, jb, g);
        }
    });
}

hipError_t launch_pairs_grad(const PairJob* jobs, int njobs, int precision, double alpha,
                             double beta, hipStream_t s)
{
    const dim3 block(kBlock);
    const bool p6 = is_p6(alpha, beta);
    const PowGen g = make_gen(alpha, beta);
    return for_each_batch(jobs, njobs, [&](const PairBatch& jb, dim3 grid) {
        if (precision == TP_PREC_FP64) {
            if (p6) hipLaunchKernelGGL(k_grad64<PowP6>, grid, block, 0, s, jb, alpha, beta, PowP6{});
            else hipLaunchKernelGGL(k_grad64<PowGen>, grid, block, 0, s, jb, alpha, beta, g);
        } else if (precision == TP_PREC_FP32_NEAR64) {
            if (p6) hipLaunchKernelGGL((k_grad32<kNiGrad32, true, true, PowP6>), grid, block, 0, s, jb, alpha, beta, PowP6{});
            else hipLaunchKernelGGL((k_grad32<kNiGrad32, true, true, PowGen>), grid, block, 0, s, jb, alpha, beta, g);
        } else if (precision == TP_PREC_FP32_ACC32) {
            if (p6) hipLaunchKernelGGL((k_grad32<kNiGrad32, false, false, PowP6, kAcc32>), grid, block, 0, s, jb, alpha, beta, PowP6{});
            else hipLaunchKernelGGL((k_grad32<kNiGrad32, false, false, PowGen, kAcc32>), grid, block, 0, s, jb, alpha, beta, g);
        } else if (precision == TP_PREC_FP32_KAHAN) {
            if (p6) hipLaunchKernelGGL((k_grad32<kNiGrad32, false, false, PowP6, kAccKahan>), grid, block, 0, s, jb, alpha, beta, PowP6{});
            else hipLaunchKernelGGL((k_grad32<kNiGrad32, false, false, PowGen, kAccKahan>), grid, block, 0, s, jb, alpha, beta, g);
        } else if (precision == TP_PREC_FP32_HILO) {
            if (p6) hipLaunchKernelGGL((k_grad32<kNiGrad32, true, false, PowP6>), grid, block, 0, s, jb, alpha, beta, PowP6{});
            else hipLaunchKernelGGL((k_grad32<kNiGrad32, true, false, PowGen>), grid, block, 0, s, jb, alpha, beta, g);
        } else {
            if (p6) hipLaunchKernelGGL((k_grad32<kNiGrad32, false, false, PowP6>), grid, block, 0, s, jb, alpha, beta, PowP6{});
            else hipLaunchKernelGGL((k_grad32<kNiGrad32, false, false, PowGen>), grid, block, 0, s, jb, alpha, beta, g);
        }
    });
}

template <int KC>
static hipError_t launch_frac_k(const PairJob* jobs, int njobs, int precision, double expo,
                                hipStream_t s)
{
    const dim3 block(kBlock);
    return for_each_batch(jobs, njobs, [&](const PairBatch& jb, dim3 grid) {
        if (precision == TP_PREC_FP64)
            hipLaunchKernelGGL(k_frac64<KC>, grid, block, 0, s, jb, expo);
        else if (precision == TP_PREC_FP32_HILO || precision == TP_PREC_FP32_NEAR64)
            hipLaunchKernelGGL((k_frac32<kNiFrac32, KC, true>), grid, block, 0, s, jb, (float)expo);
        else
            hipLaunchKernelGGL((k_frac32<kNiFrac32, KC, false>), grid, block, 0, s, jb, (float)expo);
    });
}

int frac_sym_block_faces() { return kSymFaces; }

static int64_t sym_blocks(int64_t nF) { return (nF + kSymFaces - 1) / kSymFaces; }

size_t sym_part_floats(int64_t nF, int kc, int K)
{
    const int64_t nB = sym_blocks(nF), ldp = nB * kSymFaces;
    if (K >= nB) return (size_t)nB * (size_t)kc * (size_t)ldp;        // one array [nB][kc][ldp]
    return 2 * (size_t)K * (size_t)kc * (size_t)ldp;                  // [K][kc][ldp] + [nB][kc][K blk]
}

int sym_band_blocks(int64_t nF, int kc, double max_bytes)
{
    const int64_t nB = std::max<int64_t>(1, sym_blocks(nF));
    if (4.0 * (double)sym_part_floats(nF, kc, (int)nB) <= max_bytes) return (int)nB;
    const double per = 4.0 * 2.0 * (double)kc * (double)(nB * kSymFaces);   // bytes per block of height
    return (int)std::max<double>(1.0, std::min<double>((double)nB, std::floor(max_bytes / per)));
}

int64_t sym_band_units(int64_t nF, int a0, int a1)
{
    return sym_band_offdiag((int)sym_blocks(nF), a0, a1) + (a1 - a0);
}

void sym_regions(float* part, int64_t nF, int kc, int K, float*& partT, float*& partS, int64_t& ldp, int64_t& ldS)
{
    const int64_t nB = sym_blocks(nF);
    ldp = nB * kSymFaces;
    partT = part;
    if (K >= nB) {
        partS = part;
        ldS = ldp;
    } else {
        partS = part + (size_t)K * (size_t)kc * (size_t)ldp;
        ldS = (int64_t)K * kSymFaces;
    }
}

template <int KC>
static void launch_frac_sym_k(const SymFracArgs& A, bool hilo, float expo, dim3 grid, hipStream_t s)
{
    if (hilo) hipLaunchKernelGGL((k_frac32_sym<KC, true>), grid, dim3(kBlock), 0, s, A, expo);
    else hipLaunchKernelGGL((k_frac32_sym<KC, false>), grid, dim3(kBlock), 0, s, A, expo);
}

hipError_t launch_frac_sym(const FaceData& fd, const float* ub, float* part, int K, int a0, int a1, int precision,
                           double sigma, int kc, hipStream_t s)
{
    if (fd.nF < 1) return hipSuccess;
    if (kc < 1 || kc > 9 || precision == TP_PREC_FP64 || !fd.tbox) return hipErrorInvalidValue;
    SymFracArgs A;
    A.fx = fd.fx;
    A.fl = fd.fl;
    A.ub = ub;
    A.tbox = fd.tbox;
    A.nB = (int)sym_blocks(fd.nF);
    if (K < 1 || a0 < 0 || a1 <= a0 || a1 > A.nB || a1 - a0 > K) return hipErrorInvalidValue;
    sym_regions(part, fd.nF, kc, K, A.part, A.partS, A.ldp, A.ldS);
    A.a0 = a0;
    A.a1 = a1;
    // the blocks read faces [0, ldp) of arrays of cap entries
    if (A.ldp > fd.cap) return hipErrorInvalidValue;
    const int64_t units = sym_band_units(fd.nF, a0, a1);
    const int64_t blocks = (units + kBlock / 64 - 1) / (kBlock / 64);
    if (blocks > (int64_t)INT32_MAX) return hipErrorInvalidValue;
    const dim3 grid((unsigned)blocks);
    const float expo = (float)(-(2.0 * sigma + 2.0) * 0.5);   // |d|^-(2 sigma + 2) = r2^expo
    const bool hilo = precision == TP_PREC_FP32_HILO || precision == TP_PREC_FP32_NEAR64;
    switch (kc) {
    case 1: launch_frac_sym_k<1>(A, hilo, expo, grid, s); break;
    case 2: launch_frac_sym_k<2>(A, hilo, expo, grid, s); break;
    case 3: launch_frac_sym_k<3>(A, hilo, expo, grid, s); break;
    case 4: launch_frac_sym_k<4>(A, hilo, expo, grid, s); break;
    case 5: launch_frac_sym_k<5>(A, hilo, expo, grid, s); break;
    case 6: launch_frac_sym_k<6>(A, hilo, expo, grid, s); break;
    case 7: launch_frac_sym_k<7>(A, hilo, expo, grid, s); break;
    case 8: launch_frac_sym_k<8>(A, hilo, expo, grid, s); break;
    default: launch_frac_sym_k<9>(A, hilo, expo, grid, s); break;
    }
    return hipGetLastError();
}

hipError_t launch_reduce_sym_band(const float* part, int64_t nF, int kc, int K, int a0, int a1, const double* extra,
                                  double* out, int64_t out_stride, hipStream_t s)
{
    const int nB = (int)sym_blocks(nF);
    if (nF < 1 || kc < 1) return hipSuccess;
    if (K < 1 || a0 < 0 || a1 <= a0 || a1 > nB || a1 - a0 > K) return hipErrorInvalidValue;
    float *partT, *partS;
    int64_t ldp, ldS;
    sym_regions(const_cast<float*>(part), nF, kc, K, partT, partS, ldp, ldS);
    const int64_t total = (nF - (int64_t)a0 * kSymFaces) * kc;
    if (total <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_reduce_sym_band, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, partT, partS, nB,
                       a0, a1, kc, ldp, ldS, nF, extra, out, out_stride);
    return hipGetLastError();
}

hipError_t launch_grad_sym(const FaceData& fd, float* part, int K, int a0, int a1, int precision, double alpha,
                           double beta, float rho2, hipStream_t s)
{
    if (fd.nF < 1) return hipSuccess;
    if (precision == TP_PREC_FP64 || !fd.tbox) return hipErrorInvalidValue;
    GSymArgs A;
    A.fx = fd.fx;
    A.fl = fd.fl;
    A.fn = fd.fn;
    A.dx = fd.dx;
    A.dn = fd.dn;
    A.tbox = fd.tbox;
    A.nB = (int)sym_blocks(fd.nF);
    if (K < 1 || a0 < 0 || a1 <= a0 || a1 > A.nB || a1 - a0 > K) return hipErrorInvalidValue;
    sym_regions(part, fd.nF, kGradOut, K, A.part, A.partS, A.ldp, A.ldS);
    A.a0 = a0;
    A.a1 = a1;
    A.rho2 = rho2;
    if (A.ldp > fd.cap) return hipErrorInvalidValue;
    const int64_t units = sym_band_units(fd.nF, a0, a1);
    const int64_t blocks = (units + kBlock / 64 - 1) / (kBlock / 64);
    if (blocks > (int64_t)INT32_MAX) return hipErrorInvalidValue;
    const dim3 grid((unsigned)blocks), block(kBlock);
    const bool hilo = precision == TP_PREC_FP32_HILO || precision == TP_PREC_FP32_NEAR64;
    const bool near = precision == TP_PREC_FP32_NEAR64;
    if (is_p6(alpha, beta)) {
        const PowP6 pw;
        if (near) hipLaunchKernelGGL((k_grad32_sym<true, true, PowP6>), grid, block, 0, s, A, alpha, beta, pw);
        else if (hilo) hipLaunchKernelGGL((k_grad32_sym<true, false, PowP6>), grid, block, 0, s, A, alpha, beta, pw);
        else hipLaunchKernelGGL((k_grad32_sym<false, false, PowP6>), grid, block, 0, s, A, alpha, beta, pw);
    } else {
        const PowGen pw = make_gen(alpha, beta);
        if (near) hipLaunchKernelGGL((k_grad32_sym<true, true, PowGen>), grid, block, 0, s, A, alpha, beta, pw);
        else if (hilo) hipLaunchKernelGGL((k_grad32_sym<true, false, PowGen>), grid, block, 0, s, A, alpha, beta, pw);
        else hipLaunchKernelGGL((k_grad32_sym<false, false, PowGen>), grid, block, 0, s, A, alpha, beta, pw);
    }
    return hipGetLastError();
}

int64_t sym_units(int64_t nF) { return sym_band_units(nF, 0, (int)sym_blocks(nF)); }

hipError_t launch_energy_sym(const FaceData& fd, double* upart, int precision, double alpha, double beta, float rho2,
                             hipStream_t s)
{
    if (fd.nF < 1) return hipSuccess;
    if (precision == TP_PREC_FP64 || !fd.tbox) return hipErrorInvalidValue;
    ESymArgs A;
    A.fx = fd.fx;
    A.fl = fd.fl;
    A.fn = fd.fn;
    A.tbox = fd.tbox;
    A.upart = upart;
    A.nF = fd.nF;
    A.nB = (int)sym_blocks(fd.nF);
    A.rho2 = rho2;
    if ((int64_t)A.nB * kSymFaces > fd.cap) return hipErrorInvalidValue;
    const int64_t units = sym_units(fd.nF);
    const int64_t blocks = (units + kBlock / 64 - 1) / (kBlock / 64);
    if (blocks > (int64_t)INT32_MAX) return hipErrorInvalidValue;
    const dim3 grid((unsigned)blocks), block(kBlock);
    const bool hilo = precision == TP_PREC_FP32_HILO || precision == TP_PREC_FP32_NEAR64;
    const bool near = precision == TP_PREC_FP32_NEAR64;
    if (is_p6(alpha, beta)) {
        const PowP6 pw;
        if (near) hipLaunchKernelGGL((k_energy32_sym<true, true, PowP6>), grid, block, 0, s, A, pw);
        else if (hilo) hipLaunchKernelGGL((k_energy32_sym<true, false, PowP6>), grid, block, 0, s, A, pw);
        else hipLaunchKernelGGL((k_energy32_sym<false, false, PowP6>), grid, block, 0, s, A, pw);
    } else {
        const PowGen pw = make_gen(alpha, beta);
        if (near) hipLaunchKernelGGL((k_energy32_sym<true, true, PowGen>), grid, block, 0, s, A, pw);
        else if (hilo) hipLaunchKernelGGL((k_energy32_sym<true, false, PowGen>), grid, block, 0, s, A, pw);
        else hipLaunchKernelGGL((k_energy32_sym<false, false, PowGen>), grid, block, 0, s, A, pw);
    }
    return hipGetLastError();
}

hipError_t launch_area_times(const FaceData& fd, const double* near, int64_t n, double* out, hipStream_t s)
{
    if (n < 1) return hipSuccess;
    hipLaunchKernelGGL(k_area_times, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, fd.dx, near, n, out);
    return hipGetLastError();
}

int near_block_faces() { return kNearFaces; }

int near_grid_gmax(int64_t nF)
{
    int g = (int)std::floor(std::cbrt(8.0 * (double)std::max<int64_t>(nF, 1)));
    return std::max(1, std::min(128, g));
}

static int near_key_bits(int gmax)
{
    const int64_t cells = (int64_t)gmax * gmax * gmax;
    int b = 1;
    while (((int64_t)1 << b) < cells) ++b;
    return b;
}

size_t near_grid_sort_temp_bytes(int64_t nF)
{
    size_t bytes = 0;
    (void)hipcub::DeviceRadixSort::SortPairs(nullptr, bytes, (const uint32_t*)nullptr, (uint32_t*)nullptr,
                                             (const int32_t*)nullptr, (int32_t*)nullptr, (int)std::max<int64_t>(nF, 1),
                                             0, near_key_bits(near_grid_gmax(nF)));
    return bytes;
}

hipError_t launch_near_grid_build(const NearGrid& g, const FaceData& fd, int64_t nF, float rho2, hipStream_t s)
{
    if (nF < 1) return hipSuccess;
    hipLaunchKernelGGL(k_near_grid_params, dim3(1), dim3(256), 0, s, fd.tbox, (int)(fd.cap / kTileJ), nF, rho2,
                       g.gmax, g.prm);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const unsigned nb = (unsigned)((nF + 255) / 256);
    hipLaunchKernelGGL(k_near_grid_keys, dim3(nb), dim3(256), 0, s, fd.fx, nF, g.prm, g.kin, g.vin);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    size_t bytes = g.sort_bytes;
    e = hipcub::DeviceRadixSort::SortPairs(g.sort_tmp, bytes, g.kin, g.kout, g.vin, g.vout, (int)nF, 0,
                                           near_key_bits(g.gmax), s);
    if (e != hipSuccess) return e;
    const int64_t ncell = (int64_t)g.gmax * g.gmax * g.gmax;
    hipLaunchKernelGGL(k_near_grid_clear, dim3((unsigned)((ncell + 255) / 256)), dim3(256), 0, s, g.cell, ncell);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_near_grid_mark, dim3(nb), dim3(256), 0, s, g.kout, g.vout, nF, fd.fx, fd.fl, g.cell, g.sfx,
                       g.sfl);
    return hipGetLastError();
}

hipError_t launch_near64(const PairJob* jobs, int njobs, double alpha, double beta, bool grad, hipStream_t s)
{
    const dim3 block(kNearBlock);
    const bool gen = !is_p6(alpha, beta);
    return for_each_batch(jobs, njobs, [&](const PairBatch& jb, dim3 grid) {
        if (grad) {
            if (gen) hipLaunchKernelGGL((k_near64<true, true>), grid, block, 0, s, jb, alpha, beta);
            else hipLaunchKernelGGL((k_near64<false, true>), grid, block, 0, s, jb, alpha, beta);
        } else {
            if (gen) hipLaunchKernelGGL((k_near64<true, false>), grid, block, 0, s, jb, alpha, beta);
            else hipLaunchKernelGGL((k_near64<false, false>), grid, block, 0, s, jb, alpha, beta);
        }
    });
}

hipError_t launch_pairs_frac(const PairJob* jobs, int njobs, int precision, double sigma, int k,
                             hipStream_t s)
{
    const double expo = -(2.0 * sigma + 2.0) * 0.5;   // |d|^-(2 sigma + 2) = r2^expo
    switch (k) {
    case 1: return launch_frac_k<1>(jobs, njobs, precision, expo, s);
    case 2: return launch_frac_k<2>(jobs, njobs, precision, expo, s);
    case 3: return launch_frac_k<3>(jobs, njobs, precision, expo, s);
    case 4: return launch_frac_k<4>(jobs, njobs, precision, expo, s);
    case 5: return launch_frac_k<5>(jobs, njobs, precision, expo, s);
    case 6: return launch_frac_k<6>(jobs, njobs, precision, expo, s);
    case 7: return launch_frac_k<7>(jobs, njobs, precision, expo, s);
    case 8: return launch_frac_k<8>(jobs, njobs, precision, expo, s);
    case 9: return launch_frac_k<9>(jobs, njobs, precision, expo, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace tp
