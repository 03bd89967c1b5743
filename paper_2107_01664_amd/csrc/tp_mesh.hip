// Per-face, per-vertex and sparse kernels: face geometry, vertex-face incidence, cotan
// stiffness matrix, chain rule from faces to vertices, deterministic reductions.
// All of these are O(F) or O(nnz) passes bounded by memory traffic; they use FP64.
#include "tp_internal.h"

namespace tp {

namespace {
inline unsigned nblocks(int64_t n, int b = 256) { return (unsigned)((n + b - 1) / b); }
}

// ------------------------------------------------------------------ face geometry
//
// X_S = (f_i + f_j + f_k)/3, c = (f_j - f_i) x (f_k - f_i), a_S = |c|/2, N_S = c/|c|
// (Sec. 3.1).  Padding entries (S >= nF) sit at 1e18 with zero area and normal.

__device__ __forceinline__ void write_face(const FaceData& fd, int64_t s, double X0, double X1,
                                           double X2, double N0, double N1, double N2, double a)
{
    const float h0 = (float)X0, h1 = (float)X1, h2 = (float)X2;
    fd.fx[s] = make_float4(h0, h1, h2, (float)a);
    fd.fl[s] = make_float4((float)(X0 - (double)h0), (float)(X1 - (double)h1),
                           (float)(X2 - (double)h2), 0.f);
    fd.fn[s] = make_float4((float)N0, (float)N1, (float)N2, 0.f);
    fd.dx[s] = make_double4(X0, X1, X2, a);
    fd.dn[s] = make_double4(N0, N1, N2, 0.0);
}

__device__ __forceinline__ void write_pad(const FaceData& fd, int64_t s)
{
    const double far = 1.0e18;
    fd.fx[s] = make_float4((float)far, (float)far, (float)far, 0.f);
    fd.fl[s] = make_float4(0.f, 0.f, 0.f, 0.f);
    fd.fn[s] = make_float4(0.f, 0.f, 0.f, 0.f);
    fd.dx[s] = make_double4(far, far, far, 0.0);
    fd.dn[s] = make_double4(0.0, 0.0, 0.0, 0.0);
}

__global__ void k_face_geom(const double* __restrict__ V, int64_t nV, const int32_t* __restrict__ F,
                            int64_t nF, FaceData fd, int* __restrict__ flags)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= fd.cap) return;
    if (s >= nF) {
        write_pad(fd, s);
        return;
    }
    const int32_t i = F[3 * s], j = F[3 * s + 1], k = F[3 * s + 2];
    if (i < 0 || j < 0 || k < 0 || i >= nV || j >= nV || k >= nV) {
        flags[kFlagBadIndex] = 1;
        write_pad(fd, s);
        return;
    }
    double fi[3], fj[3], fk[3];
    for (int m = 0; m < 3; ++m) {
        fi[m] = V[3 * (int64_t)i + m];
        fj[m] = V[3 * (int64_t)j + m];
        fk[m] = V[3 * (int64_t)k + m];
    }
    double X[3], e1[3], e2[3];
    for (int m = 0; m < 3; ++m) {
        X[m] = (fi[m] + fj[m] + fk[m]) / 3.0;
        e1[m] = fj[m] - fi[m];
        e2[m] = fk[m] - fi[m];
    }
    const double c0 = e1[1] * e2[2] - e1[2] * e2[1];
    const double c1 = e1[2] * e2[0] - e1[0] * e2[2];
    const double c2 = e1[0] * e2[1] - e1[1] * e2[0];
    const double cn = sqrt(c0 * c0 + c1 * c1 + c2 * c2);
    if (!isfinite(cn) || !isfinite(X[0] + X[1] + X[2])) {
        flags[kFlagNonFinite] = 1;
        write_pad(fd, s);
        return;
    }
    if (!(cn > 1e-300) || (float)(0.5 * cn) == 0.0f) {
        flags[kFlagDegenerate] = 1;
        write_pad(fd, s);
        return;
    }
    write_face(fd, s, X[0], X[1], X[2], c0 / cn, c1 / cn, c2 / cn, 0.5 * cn);
}

// Boxes of the FP32 barycenters (hi parts) of the real faces of every tile of kTileJ
// faces; a tile of padding faces gets an empty box (lo = +inf, hi = -inf).
__global__ __launch_bounds__(kTileJ) void k_tile_boxes(FaceData fd)
{
    __shared__ float sh[6][kTileJ];
    const int64_t s = (int64_t)blockIdx.x * kTileJ + threadIdx.x;
    float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    if (s < fd.nF) {
        const float4 x = fd.fx[s];
        lo[0] = hi[0] = x.x;
        lo[1] = hi[1] = x.y;
        lo[2] = hi[2] = x.z;
    }
    for (int m = 0; m < 3; ++m) {
        sh[m][threadIdx.x] = lo[m];
        sh[3 + m][threadIdx.x] = hi[m];
    }
    __syncthreads();
    for (int w = kTileJ / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int m = 0; m < 3; ++m) {
                sh[m][threadIdx.x] = fminf(sh[m][threadIdx.x], sh[m][threadIdx.x + w]);
                sh[3 + m][threadIdx.x] = fmaxf(sh[3 + m][threadIdx.x], sh[3 + m][threadIdx.x + w]);
            }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        fd.tbox[2 * blockIdx.x] = make_float4(sh[0][0], sh[1][0], sh[2][0], 0.f);
        fd.tbox[2 * blockIdx.x + 1] = make_float4(sh[3][0], sh[4][0], sh[5][0], 0.f);
    }
}

static hipError_t launch_tile_boxes(const FaceData& fd, hipStream_t s)
{
    if (!fd.tbox) return hipSuccess;
    hipLaunchKernelGGL(k_tile_boxes, dim3((unsigned)(fd.cap / kTileJ)), dim3(kTileJ), 0, s, fd);
    return hipGetLastError();
}

hipError_t launch_face_geom(const double* V, int64_t nV, const int32_t* F, int64_t nF,
                            const FaceData& fd, int* flags, hipStream_t s)
{
    hipLaunchKernelGGL(k_face_geom, dim3(nblocks(fd.cap)), dim3(256), 0, s, V, nV, F, nF, fd, flags);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_tile_boxes(fd, s);
}

__global__ void k_face_from_quantities(const double* __restrict__ X, const double* __restrict__ N,
                                       const double* __restrict__ a, int64_t nF, FaceData fd,
                                       int* __restrict__ flags)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= fd.cap) return;
    if (s >= nF) {
        write_pad(fd, s);
        return;
    }
    const double x0 = X[3 * s], x1 = X[3 * s + 1], x2 = X[3 * s + 2];
    const double n0 = N[3 * s], n1 = N[3 * s + 1], n2 = N[3 * s + 2];
    const double as = a[s];
    if (!isfinite(x0 + x1 + x2 + n0 + n1 + n2 + as)) {
        flags[kFlagNonFinite] = 1;
        write_pad(fd, s);
        return;
    }
    write_face(fd, s, x0, x1, x2, n0, n1, n2, as);
}

hipError_t launch_face_from_quantities(const double* X, const double* N, const double* a,
                                       int64_t nF, const FaceData& fd, int* flags, hipStream_t s)
{
    hipLaunchKernelGGL(k_face_from_quantities, dim3(nblocks(fd.cap)), dim3(256), 0, s, X, N, a, nF, fd, flags);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_tile_boxes(fd, s);
}

// ------------------------------------------------------------------ vertex-face incidence
//
// CSR of (face, corner) entries per vertex, entry = 3 * face + corner, sorted within each
// row, so every gather over it has a fixed order.  Integer atomics only place entries;
// the per-row sort makes the result independent of their order.

// Index check: every face corner must name a vertex in [0, nV).
__global__ void k_check_indices(const int32_t* __restrict__ F, int64_t n3, int64_t nV,
                                int* __restrict__ flags)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n3 && (F[t] < 0 || F[t] >= nV)) flags[kFlagBadIndex] = 1;
}

hipError_t launch_check_indices(const int32_t* F, int64_t nF, int64_t nV, int* flags, hipStream_t s)
{
    hipLaunchKernelGGL(k_check_indices, dim3(nblocks(3 * nF)), dim3(256), 0, s, F, 3 * nF, nV, flags);
    return hipGetLastError();
}

__global__ void k_vf_count(const int32_t* __restrict__ F, int64_t n3, int64_t nV, int32_t* deg)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n3 && F[t] >= 0 && F[t] < nV) atomicAdd(&deg[F[t]], 1);
}

hipError_t launch_vf_count(const int32_t* F, int64_t nF, int64_t nV, int32_t* deg, hipStream_t s)
{
    hipLaunchKernelGGL(k_vf_count, dim3(nblocks(3 * nF)), dim3(256), 0, s, F, 3 * nF, nV, deg);
    return hipGetLastError();
}

// Exclusive scan by one workgroup of 1024 threads: each thread owns a contiguous segment.
__global__ __launch_bounds__(1024) void k_scan(const int32_t* __restrict__ in, int64_t n,
                                               int32_t* __restrict__ out)
{
    __shared__ int64_t sums[1024];
    const int t = threadIdx.x;
    const int64_t seg = (n + 1023) / 1024;
    const int64_t b = t * seg, e = min(n, b + seg);
    int64_t acc = 0;
    for (int64_t i = b; i < e; ++i) acc += in[i];
    sums[t] = acc;
    __syncthreads();
    if (t == 0) {
        int64_t run = 0;
        for (int q = 0; q < 1024; ++q) {
            int64_t v = sums[q];
            sums[q] = run;
            run += v;
        }
        out[n] = (int32_t)run;
    }
    __syncthreads();
    int64_t run = sums[t];
    for (int64_t i = b; i < e; ++i) {
        out[i] = (int32_t)run;
        run += in[i];
    }
}

hipError_t launch_scan(const int32_t* in, int64_t n, int32_t* out_excl, hipStream_t s)
{
    hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, s, in, n, out_excl);
    return hipGetLastError();
}

__global__ void k_vf_fill(const int32_t* __restrict__ F, int64_t n3, int64_t nV,
                          const int32_t* __restrict__ off, int32_t* cursor, int32_t* __restrict__ idx)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n3) return;
    const int32_t v = F[t];
    if (v < 0 || v >= nV) return;
    const int32_t pos = off[v] + atomicAdd(&cursor[v], 1);
    idx[pos] = (int32_t)t;   // t = 3 * face + corner
}

hipError_t launch_vf_fill(const int32_t* F, int64_t nF, int64_t nV, const int32_t* off,
                          int32_t* cursor, int32_t* idx, hipStream_t s)
{
    hipLaunchKernelGGL(k_vf_fill, dim3(nblocks(3 * nF)), dim3(256), 0, s, F, 3 * nF, nV, off, cursor, idx);
    return hipGetLastError();
}

__global__ void k_sort_rows(const int32_t* __restrict__ off, int64_t n, int32_t* __restrict__ idx)
{
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    const int32_t b = off[v], e = off[v + 1];
    for (int32_t i = b + 1; i < e; ++i) {
        const int32_t key = idx[i];
        int32_t j = i - 1;
        while (j >= b && idx[j] > key) {
            idx[j + 1] = idx[j];
            --j;
        }
        idx[j + 1] = key;
    }
}

hipError_t launch_sort_rows(const int32_t* off, int64_t n, int32_t* idx, hipStream_t s)
{
    hipLaunchKernelGGL(k_sort_rows, dim3(nblocks(n)), dim3(256), 0, s, off, n, idx);
    return hipGetLastError();
}

// ------------------------------------------------------------------ cotan stiffness matrix
//
// Pattern: for vertex v, the other two corners of every incident face, sorted and made
// unique, plus v itself.  cand holds 2 entries per incidence at 2 * vf_off[v].

__global__ void k_lap_count(const int32_t* __restrict__ F, int64_t nV,
                            const int32_t* __restrict__ vf_off, const int32_t* __restrict__ vf_idx,
                            int32_t* __restrict__ cand, int32_t* __restrict__ cnt)
{
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= nV) return;
    const int32_t b = vf_off[v], e = vf_off[v + 1];
    int32_t* c = cand + 2 * (int64_t)b;
    int32_t m = 0;
    for (int32_t q = b; q < e; ++q) {
        const int32_t ent = vf_idx[q];
        const int32_t f = ent / 3, corner = ent - 3 * f;
        c[m++] = F[3 * (int64_t)f + (corner + 1) % 3];
        c[m++] = F[3 * (int64_t)f + (corner + 2) % 3];
    }
    for (int32_t i = 1; i < m; ++i) {          // insertion sort (rows are short)
        const int32_t key = c[i];
        int32_t j = i - 1;
        while (j >= 0 && c[j] > key) {
            c[j + 1] = c[j];
            --j;
        }
        c[j + 1] = key;
    }
    int32_t u = 0;
    for (int32_t i = 0; i < m; ++i)
        if (i == 0 || c[i] != c[i - 1]) ++u;
    cnt[v] = u + 1;   // + diagonal
}

hipError_t launch_lap_pattern_count(const int32_t* F, int64_t nV, const int32_t* vf_off,
                                    const int32_t* vf_idx, int32_t* cand, int32_t* cnt,
                                    hipStream_t s)
{
    hipLaunchKernelGGL(k_lap_count, dim3(nblocks(nV)), dim3(256), 0, s, F, nV, vf_off, vf_idx, cand, cnt);
    return hipGetLastError();
}

__global__ void k_lap_fill(int64_t nV, const int32_t* __restrict__ vf_off,
                           const int32_t* __restrict__ cand, const int32_t* __restrict__ lap_off,
                           int32_t* __restrict__ lap_col)
{
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= nV) return;
    const int32_t m = 2 * (vf_off[v + 1] - vf_off[v]);
    const int32_t* c = cand + 2 * (int64_t)vf_off[v];
    int32_t* out = lap_col + lap_off[v];
    int32_t w = 0;
    bool diag_done = false;
    for (int32_t i = 0; i < m; ++i) {
        if (i > 0 && c[i] == c[i - 1]) continue;
        if (!diag_done && c[i] > v) {
            out[w++] = (int32_t)v;
            diag_done = true;
        }
        out[w++] = c[i];
    }
    if (!diag_done) out[w++] = (int32_t)v;
}

hipError_t launch_lap_pattern_fill(int64_t nV, const int32_t* vf_off, const int32_t* cand,
                                   const int32_t* lap_off, int32_t* lap_col, hipStream_t s)
{
    hipLaunchKernelGGL(k_lap_fill, dim3(nblocks(nV)), dim3(256), 0, s, nV, vf_off, cand, lap_off, lap_col);
    return hipGetLastError();
}

__device__ __forceinline__ double cot_at(const double* a, const double* b, const double* c)
{
    // cotangent of the angle at corner a of triangle (a, b, c)
    const double u0 = b[0] - a[0], u1 = b[1] - a[1], u2 = b[2] - a[2];
    const double w0 = c[0] - a[0], w1 = c[1] - a[1], w2 = c[2] - a[2];
    const double dot = u0 * w0 + u1 * w1 + u2 * w2;
    const double x0 = u1 * w2 - u2 * w1, x1 = u2 * w0 - u0 * w2, x2 = u0 * w1 - u1 * w0;
    return dot / sqrt(x0 * x0 + x1 * x1 + x2 * x2);
}

__device__ __forceinline__ int32_t find_col(const int32_t* col, int32_t b, int32_t e, int32_t key)
{
    for (int32_t q = b; q < e; ++q)
        if (col[q] == key) return q;
    return -1;
}

// Row v of C: for each incident face (v, j, k) (cyclic from v), the angle at k is opposite
// edge vj and the angle at j is opposite edge vk:
//   C_vj -= cot_k / 2,  C_vk -= cot_j / 2,  C_vv += (cot_j + cot_k) / 2.
__global__ void k_cotan(const double* __restrict__ V, const int32_t* __restrict__ F, int64_t nV,
                        const int32_t* __restrict__ vf_off, const int32_t* __restrict__ vf_idx,
                        const int32_t* __restrict__ lap_off, const int32_t* __restrict__ lap_col,
                        double* __restrict__ lap_val)
{
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= nV) return;
    const int32_t b = lap_off[v], e = lap_off[v + 1];
    for (int32_t q = b; q < e; ++q) lap_val[q] = 0.0;
    const int32_t dq = find_col(lap_col, b, e, (int32_t)v);
    double diag = 0.0;
    for (int32_t q = vf_off[v]; q < vf_off[v + 1]; ++q) {
        const int32_t ent = vf_idx[q];
        const int32_t f = ent / 3, corner = ent - 3 * f;
        const int32_t j = F[3 * (int64_t)f + (corner + 1) % 3];
        const int32_t k = F[3 * (int64_t)f + (corner + 2) % 3];
        const double* pv = V + 3 * v;
        const double* pj = V + 3 * (int64_t)j;
        const double* pk = V + 3 * (int64_t)k;
        const double cj = cot_at(pj, pk, pv), ck = cot_at(pk, pv, pj);
        const int32_t qj = find_col(lap_col, b, e, j), qk = find_col(lap_col, b, e, k);
        if (qj >= 0) lap_val[qj] -= 0.5 * ck;
        if (qk >= 0) lap_val[qk] -= 0.5 * cj;
        diag += 0.5 * (cj + ck);
    }
    if (dq >= 0) lap_val[dq] += diag;
}

hipError_t launch_cotan_values(const double* V, const int32_t* F, int64_t nV,
                               const int32_t* vf_off, const int32_t* vf_idx,
                               const int32_t* lap_off, const int32_t* lap_col, double* lap_val,
                               hipStream_t s)
{
    hipLaunchKernelGGL(k_cotan, dim3(nblocks(nV)), dim3(256), 0, s, V, F, nV, vf_off, vf_idx, lap_off, lap_col, lap_val);
    return hipGetLastError();
}

// ------------------------------------------------------------------ chain rule to vertices
//
// gface rows (stride gstride): dE/dX (3), dE/dN (3), dE/da (1) per face.  For face
// (i,j,k) with e1 = f_j - f_i, e2 = f_k - f_i, c = e1 x e2:
//   g_c = (I - N N^T) dE/dN / |c| + dE/da N / 2,
//   d/df_j = e2 x g_c,  d/df_k = g_c x e1,  d/df_i = -(d/df_j + d/df_k),
// and each corner also receives dE/dX / 3.

__global__ void k_grad_gather(const double* __restrict__ V, const int32_t* __restrict__ F,
                              int64_t nV, const int32_t* __restrict__ vf_off,
                              const int32_t* __restrict__ vf_idx, const double* __restrict__ g,
                              int64_t gs, double* __restrict__ dE)
{
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= nV) return;
    double o0 = 0.0, o1 = 0.0, o2 = 0.0;
    for (int32_t q = vf_off[v]; q < vf_off[v + 1]; ++q) {
        const int32_t ent = vf_idx[q];
        const int64_t f = ent / 3;
        const int corner = ent - 3 * (int)f;
        const double* fi = V + 3 * (int64_t)F[3 * f];
        const double* fj = V + 3 * (int64_t)F[3 * f + 1];
        const double* fk = V + 3 * (int64_t)F[3 * f + 2];
        const double e10 = fj[0] - fi[0], e11 = fj[1] - fi[1], e12 = fj[2] - fi[2];
        const double e20 = fk[0] - fi[0], e21 = fk[1] - fi[1], e22 = fk[2] - fi[2];
        const double c0 = e11 * e22 - e12 * e21, c1 = e12 * e20 - e10 * e22, c2 = e10 * e21 - e11 * e20;
        const double cn = sqrt(c0 * c0 + c1 * c1 + c2 * c2);
        const double n0 = c0 / cn, n1 = c1 / cn, n2 = c2 / cn;
        const double gx0 = g[f], gx1 = g[gs + f], gx2 = g[2 * gs + f];
        const double gn0 = g[3 * gs + f], gn1 = g[4 * gs + f], gn2 = g[5 * gs + f];
        const double ga = g[6 * gs + f];
        const double ndg = n0 * gn0 + n1 * gn1 + n2 * gn2;
        const double gc0 = (gn0 - n0 * ndg) / cn + 0.5 * ga * n0;
        const double gc1 = (gn1 - n1 * ndg) / cn + 0.5 * ga * n1;
        const double gc2 = (gn2 - n2 * ndg) / cn + 0.5 * ga * n2;
        double d0, d1, d2;
        if (corner == 1) {            // e2 x g_c
            d0 = e21 * gc2 - e22 * gc1; d1 = e22 * gc0 - e20 * gc2; d2 = e20 * gc1 - e21 * gc0;
        } else if (corner == 2) {     // g_c x e1
            d0 = gc1 * e12 - gc2 * e11; d1 = gc2 * e10 - gc0 * e12; d2 = gc0 * e11 - gc1 * e10;
        } else {                      // -(e2 x g_c + g_c x e1)
            d0 = -((e21 * gc2 - e22 * gc1) + (gc1 * e12 - gc2 * e11));
            d1 = -((e22 * gc0 - e20 * gc2) + (gc2 * e10 - gc0 * e12));
            d2 = -((e20 * gc1 - e21 * gc0) + (gc0 * e11 - gc1 * e10));
        }
        o0 += gx0 / 3.0 + d0;
        o1 += gx1 / 3.0 + d1;
        o2 += gx2 / 3.0 + d2;
    }
    dE[3 * v] = o0;
    dE[3 * v + 1] = o1;
    dE[3 * v + 2] = o2;
}

hipError_t launch_grad_gather(const double* V, const int32_t* F, int64_t nV, int64_t nF,
                              const int32_t* vf_off, const int32_t* vf_idx,
                              const double* gface, int64_t gstride, double* dE, hipStream_t s)
{
    (void)nF;
    hipLaunchKernelGGL(k_grad_gather, dim3(nblocks(nV)), dim3(256), 0, s, V, F, nV, vf_off, vf_idx, gface, gstride, dE);
    return hipGetLastError();
}

// ------------------------------------------------------------------ fractional apply I/O
//
// ubar(S) = (u_i + u_j + u_k) / 3 per column (phi_i(S) = 1/3, Sec. 2.4), stored with row
// stride kp (FP32 or FP64); padding rows are zero.

template <class T>
__global__ void k_face_avg(const int32_t* __restrict__ F, int64_t nF, int64_t cap,
                           const double* __restrict__ u, int ldu, int k, int kp, T* __restrict__ ub)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= cap * kp) return;
    const int64_t s = t / kp;
    const int c = (int)(t - s * kp);
    T val = (T)0;
    if (s < nF && c < k) {
        const double m = (u[(int64_t)F[3 * s] * ldu + c] + u[(int64_t)F[3 * s + 1] * ldu + c] +
                          u[(int64_t)F[3 * s + 2] * ldu + c]) / 3.0;
        val = (T)m;
    }
    ub[t] = val;
}

hipError_t launch_face_avg(const int32_t* F, int64_t nF, int64_t cap, const double* u, int ldu,
                           int k, int kp, int precision, void* ub, hipStream_t s)
{
    if (precision == TP_PREC_FP64)
        hipLaunchKernelGGL(k_face_avg<double>, dim3(nblocks(cap * kp)), dim3(256), 0, s, F, nF, cap, u, ldu, k, kp, (double*)ub);
    else
        hipLaunchKernelGGL(k_face_avg<float>, dim3(nblocks(cap * kp)), dim3(256), 0, s, F, nF, cap, u, ldu, k, kp, (float*)ub);
    return hipGetLastError();
}

// (L u)_i = 2 sum_{S ni i} phi_i(S) a_S z(S) = 2 sum_{S ni i} (a_S / 3) z(S), written to
// columns [c0, c0 + k) of Lu (row stride kout).
__global__ void k_ut_gather(int64_t nV, const int32_t* __restrict__ vf_off,
                            const int32_t* __restrict__ vf_idx, const double4* __restrict__ dxa,
                            const double* __restrict__ z, int64_t zs, int k, int kout, int c0,
                            double* __restrict__ Lu)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nV * k) return;
    const int64_t v = t / k;
    const int c = (int)(t - v * k);
    double acc = 0.0;
    for (int32_t q = vf_off[v]; q < vf_off[v + 1]; ++q) {
        const int64_t f = vf_idx[q] / 3;
        acc += 2.0 * (dxa[f].w / 3.0) * z[(int64_t)c * zs + f];
    }
    Lu[v * kout + c0 + c] = acc;
}

hipError_t launch_ut_gather(const int32_t* F, int64_t nV, const int32_t* vf_off,
                            const int32_t* vf_idx, const FaceData& fd, const double* z,
                            int64_t zstride, int k, int kout, int c0, double* Lu, hipStream_t s)
{
    (void)F;
    hipLaunchKernelGGL(k_ut_gather, dim3(nblocks(nV * k)), dim3(256), 0, s, nV, vf_off, vf_idx, fd.dx, z, zstride, k, kout, c0, Lu);
    return hipGetLastError();
}

// ------------------------------------------------------------------ constraints
//
// Volume (1/6) sum_{(ijk)} f_i . (f_j x f_k) (Sec. 7.1.4); its gradient at vertex v is
// (1/6) sum over incident faces of f_j x f_k with (v, j, k) in cyclic order.

__global__ void k_volume_gradient(const double* __restrict__ V, const int32_t* __restrict__ F,
                                  int64_t nV, const int32_t* __restrict__ vf_off,
                                  const int32_t* __restrict__ vf_idx, double* __restrict__ out,
                                  int ldo, int c0)
{
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= nV) return;
    double o0 = 0.0, o1 = 0.0, o2 = 0.0;
    for (int32_t q = vf_off[v]; q < vf_off[v + 1]; ++q) {
        const int32_t ent = vf_idx[q];
        const int64_t f = ent / 3;
        const int corner = ent - 3 * (int)f;
        const double* a = V + 3 * (int64_t)F[3 * f + (corner + 1) % 3];
        const double* b = V + 3 * (int64_t)F[3 * f + (corner + 2) % 3];
        o0 += a[1] * b[2] - a[2] * b[1];
        o1 += a[2] * b[0] - a[0] * b[2];
        o2 += a[0] * b[1] - a[1] * b[0];
    }
    out[v * ldo + c0] = o0 / 6.0;
    out[v * ldo + c0 + 1] = o1 / 6.0;
    out[v * ldo + c0 + 2] = o2 / 6.0;
}

hipError_t launch_volume_gradient(const double* V, const int32_t* F, int64_t nV,
                                  const int32_t* vf_off, const int32_t* vf_idx, double* out,
                                  int ldo, int c0, hipStream_t s)
{
    hipLaunchKernelGGL(k_volume_gradient, dim3(nblocks(nV)), dim3(256), 0, s, V, F, nV, vf_off, vf_idx, out, ldo, c0);
    return hipGetLastError();
}

__global__ void k_face_volume(const double* __restrict__ V, const int32_t* __restrict__ F,
                              int64_t nF, double* __restrict__ vol6)
{
    const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= nF) return;
    const double* a = V + 3 * (int64_t)F[3 * f];
    const double* b = V + 3 * (int64_t)F[3 * f + 1];
    const double* c = V + 3 * (int64_t)F[3 * f + 2];
    vol6[f] = a[0] * (b[1] * c[2] - b[2] * c[1]) + a[1] * (b[2] * c[0] - b[0] * c[2]) +
              a[2] * (b[0] * c[1] - b[1] * c[0]);
}

hipError_t launch_face_volume(const double* V, const int32_t* F, int64_t nF, double* vol6,
                              hipStream_t s)
{
    hipLaunchKernelGGL(k_face_volume, dim3(nblocks(nF)), dim3(256), 0, s, V, F, nF, vol6);
    return hipGetLastError();
}

// ------------------------------------------------------------------ sparse times dense
// y[i, :] = sum_e val[e] x[col[e], :], k columns, one thread per (row, column).
__global__ void k_spmm(int64_t n, const int32_t* __restrict__ off, const int32_t* __restrict__ col,
                       const double* __restrict__ val, const double* __restrict__ x, int ldx, int k,
                       double* __restrict__ y, int ldy)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * k) return;
    const int64_t i = t / k;
    const int c = (int)(t - i * k);
    double acc = 0.0;
    for (int32_t e = off[i]; e < off[i + 1]; ++e) acc += val[e] * x[(int64_t)col[e] * ldx + c];
    y[i * ldy + c] = acc;
}

hipError_t launch_spmm(int64_t n, const int32_t* off, const int32_t* col, const double* val,
                       const double* x, int ldx, int k, double* y, int ldy, hipStream_t s)
{
    hipLaunchKernelGGL(k_spmm, dim3(nblocks(n * k)), dim3(256), 0, s, n, off, col, val, x, ldx, k, y, ldy);
    return hipGetLastError();
}

// ------------------------------------------------------------------ deterministic reductions
//
// Stage 1: kRedBlocks workgroups each sum a fixed contiguous chunk (thread-strided, then a
// fixed LDS tree); stage 2: one workgroup sums the kRedBlocks partials in order.  The
// partition depends only on n, so the result is reproducible bit for bit.

constexpr int kRedBlocks = 256;

size_t reduce_scratch_doubles(int ncols) { return (size_t)kRedBlocks * (size_t)ncols + 64; }

__device__ __forceinline__ double block_sum(double v, double* sh)
{
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    double r = sh[0];
    __syncthreads();
    return r;
}

__global__ __launch_bounds__(256) void k_dot_partial(const double* __restrict__ x, int ldx,
                                                     const double* __restrict__ y, int ldy,
                                                     int64_t n, int ncols,
                                                     double* __restrict__ partial)
{
    __shared__ double sh[256];
    const int64_t chunk = (n + kRedBlocks - 1) / kRedBlocks;
    const int64_t b = (int64_t)blockIdx.x * chunk, e = min(n, b + chunk);
    for (int c = 0; c < ncols; ++c) {
        double acc = 0.0;
        for (int64_t i = b + threadIdx.x; i < e; i += 256)
            acc += x[i * ldx + c] * (y ? y[i * ldy + c] : 1.0);
        const double s = block_sum(acc, sh);
        if (threadIdx.x == 0) partial[(int64_t)blockIdx.x * ncols + c] = s;
    }
}

__global__ __launch_bounds__(256) void k_dot_final(const double* __restrict__ partial, int ncols,
                                                   double* __restrict__ out)
{
    __shared__ double sh[256];
    for (int c = 0; c < ncols; ++c) {
        const double s = block_sum(partial[(int64_t)threadIdx.x * ncols + c], sh);
        if (threadIdx.x == 0) out[c] = s;
    }
}

hipError_t launch_dot_cols(const double* x, int ldx, const double* y, int ldy, int64_t n,
                           int ncols, double* scratch, double* out, hipStream_t s)
{
    static_assert(kRedBlocks == 256, "final stage sums one partial per thread");
    hipLaunchKernelGGL(k_dot_partial, dim3(kRedBlocks), dim3(256), 0, s, x, ldx, y, ldy, n, ncols, scratch);
    hipLaunchKernelGGL(k_dot_final, dim3(1), dim3(256), 0, s, scratch, ncols, out);
    return hipGetLastError();
}

__device__ __forceinline__ double block_max(double v, double* sh)
{
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + w]);
        __syncthreads();
    }
    double r = sh[0];
    __syncthreads();
    return r;
}

__global__ __launch_bounds__(256) void k_max_rownorm3(const double* __restrict__ x, int64_t n,
                                                      double* __restrict__ partial)
{
    __shared__ double sh[256];
    const int64_t chunk = (n + kRedBlocks - 1) / kRedBlocks;
    const int64_t b = (int64_t)blockIdx.x * chunk, e = min(n, b + chunk);
    double m = 0.0;
    for (int64_t i = b + threadIdx.x; i < e; i += 256)
        m = fmax(m, sqrt(x[3 * i] * x[3 * i] + x[3 * i + 1] * x[3 * i + 1] + x[3 * i + 2] * x[3 * i + 2]));
    const double r = block_max(m, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = r;
}

__global__ __launch_bounds__(256) void k_max_final(const double* __restrict__ partial,
                                                   double* __restrict__ out)
{
    __shared__ double sh[256];
    const double r = block_max(partial[threadIdx.x], sh);
    if (threadIdx.x == 0) out[0] = r;
}

hipError_t launch_max_rownorm3(const double* x, int64_t n, double* scratch, double* out,
                               hipStream_t s)
{
    hipLaunchKernelGGL(k_max_rownorm3, dim3(kRedBlocks), dim3(256), 0, s, x, n, scratch);
    hipLaunchKernelGGL(k_max_final, dim3(1), dim3(256), 0, s, scratch, out);
    return hipGetLastError();
}

// Per-component means: partial[b][comp][col] over the fixed chunk of block b, then
// mean = (sum_b partial) / count, then x -= mean[comp(v)].
size_t project_scratch_doubles(int k, int ncomp)
{
    return (size_t)kRedBlocks * (size_t)ncomp * (size_t)k + (size_t)ncomp * (size_t)k + 64;
}

__global__ __launch_bounds__(256) void k_comp_partial(const double* __restrict__ x, int ldx, int k,
                                                      int64_t n, const int32_t* __restrict__ comp,
                                                      int ncomp, double* __restrict__ partial)
{
    __shared__ double sh[256];
    const int64_t chunk = (n + kRedBlocks - 1) / kRedBlocks;
    const int64_t b = (int64_t)blockIdx.x * chunk, e = min(n, b + chunk);
    for (int cp = 0; cp < ncomp; ++cp)
        for (int c = 0; c < k; ++c) {
            double acc = 0.0;
            for (int64_t i = b + threadIdx.x; i < e; i += 256)
                if (comp[i] == cp) acc += x[i * ldx + c];
            const double s = block_sum(acc, sh);
            if (threadIdx.x == 0) partial[((int64_t)blockIdx.x * ncomp + cp) * k + c] = s;
        }
}

__global__ __launch_bounds__(256) void k_comp_final(const double* __restrict__ partial, int k,
                                                    int ncomp, const double* __restrict__ inv_count,
                                                    double* __restrict__ mean)
{
    __shared__ double sh[256];
    for (int cp = 0; cp < ncomp; ++cp)
        for (int c = 0; c < k; ++c) {
            const double s = block_sum(partial[((int64_t)threadIdx.x * ncomp + cp) * k + c], sh);
            if (threadIdx.x == 0) mean[cp * k + c] = s * inv_count[cp];
        }
}

__global__ void k_sub_mean(double* __restrict__ x, int ldx, int k, int64_t n,
                           const int32_t* __restrict__ comp, const double* __restrict__ mean)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * k) return;
    const int64_t i = t / k;
    const int c = (int)(t - i * k);
    x[i * ldx + c] -= mean[comp[i] * k + c];
}

hipError_t launch_project_mean(double* x, int ldx, int k, int64_t n, const int32_t* comp,
                               const double* inv_count, int ncomp, double* scratch,
                               hipStream_t s)
{
    double* partial = scratch;
    double* mean = scratch + (size_t)kRedBlocks * ncomp * k;
    hipLaunchKernelGGL(k_comp_partial, dim3(kRedBlocks), dim3(256), 0, s, x, ldx, k, n, comp, ncomp, partial);
    hipLaunchKernelGGL(k_comp_final, dim3(1), dim3(256), 0, s, partial, k, ncomp, inv_count, mean);
    hipLaunchKernelGGL(k_sub_mean, dim3(nblocks(n * k)), dim3(256), 0, s, x, ldx, k, n, comp, mean);
    return hipGetLastError();
}

// ------------------------------------------------------------------ small dense updates

struct Coef8 {
    double c[8];
    int col[8];
};

// out[i, 0..2] = a * x[i, 0..2] + sum_m c_m Y[i, col_m + 0..2]
__global__ void k_axpy_block3(int64_t n, const double* __restrict__ x, int ldx, double a,
                              const double* __restrict__ Y, int ldy, int ncoef, Coef8 cf,
                              double* __restrict__ out, int ldo)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * 3) return;
    const int64_t i = t / 3;
    const int c = (int)(t - i * 3);
    double v = x ? a * x[i * ldx + c] : 0.0;
    for (int m = 0; m < ncoef; ++m) v += cf.c[m] * Y[i * ldy + cf.col[m] + c];
    out[i * ldo + c] = v;
}

hipError_t launch_axpy_block3(int64_t n, const double* x, int ldx, double a,
                              const double* Y, int ldy, int ncoef, const double* coef_host,
                              const int* cols_host, double* out, int ldo, hipStream_t s)
{
    if (ncoef > 8) return hipErrorInvalidValue;
    Coef8 cf;
    for (int m = 0; m < 8; ++m) {
        cf.c[m] = m < ncoef ? coef_host[m] : 0.0;
        cf.col[m] = m < ncoef ? cols_host[m] : 0;
    }
    hipLaunchKernelGGL(k_axpy_block3, dim3(nblocks(n * 3)), dim3(256), 0, s, n, x, ldx, a, Y, ldy, ncoef, cf, out, ldo);
    return hipGetLastError();
}

__global__ void k_copy_cols(int64_t n, const double* __restrict__ x, int ldx, int k,
                            double* __restrict__ y, int ldy)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * k) return;
    const int64_t i = t / k;
    const int c = (int)(t - i * k);
    y[i * ldy + c] = x[i * ldx + c];
}

hipError_t launch_copy_cols(int64_t n, const double* x, int ldx, int k, double* y, int ldy,
                            hipStream_t s)
{
    hipLaunchKernelGGL(k_copy_cols, dim3(nblocks(n * k)), dim3(256), 0, s, n, x, ldx, k, y, ldy);
    return hipGetLastError();
}

// ------------------------------------------------------------------ vertex pins
//
// Pinned vertices (Sec. 7.1.2) enter the Poisson solves as rows appended to the Laplacian
// (Sec. 7.2): the bordered system's solution is zero at the pins and solves C x = b on the
// other rows, which is the symmetric matrix with the pinned rows and columns replaced by
// the identity and a zero right-hand side there.
__global__ void k_pin_values(int64_t n, const int32_t* __restrict__ off, const int32_t* __restrict__ col,
                             const double* __restrict__ val, const int8_t* __restrict__ pinned,
                             double* __restrict__ out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const bool pi = pinned[i] != 0;
    for (int32_t e = off[i]; e < off[i + 1]; ++e) {
        const int32_t j = col[e];
        out[e] = pi ? (j == i ? 1.0 : 0.0) : (pinned[j] ? 0.0 : val[e]);
    }
}

hipError_t launch_pin_values(int64_t n, const int32_t* off, const int32_t* col, const double* val,
                             const int8_t* pinned, double* out, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_pin_values, dim3(nblocks(n)), dim3(256), 0, s, n, off, col, val, pinned, out);
    return hipGetLastError();
}

__global__ void k_zero_pinned(double* __restrict__ x, int ldx, int k, int64_t n, const int8_t* __restrict__ pinned)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * k) return;
    const int64_t i = e / k;
    if (pinned[i]) x[i * ldx + (e - i * k)] = 0.0;
}

hipError_t launch_zero_pinned(double* x, int ldx, int k, int64_t n, const int8_t* pinned, hipStream_t s)
{
    if (n <= 0 || k <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_zero_pinned, dim3(nblocks(n * k)), dim3(256), 0, s, x, ldx, k, n, pinned);
    return hipGetLastError();
}

}  // namespace tp

