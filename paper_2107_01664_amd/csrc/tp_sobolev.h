// The inner-product operator A = B + B0 (Sec. 2.4; discrete terms in Sec. 3.2.1) applied in
// the factored form of Sec. 5.1.2 and 5.1.3.
#pragma once
#include "tp_internal.h"

namespace tp {

constexpr int kSobCols = 3;    // columns handled by one kernel instance (one coordinate each)

// Launch geometry of the pair kernel for kc columns.
PairPlan sobolev_plan(int precision, int kc, int64_t nF, int64_t cap);
// Bytes of the per-face column data (D u and ubar of kc columns, cap faces).
size_t sobolev_face_bytes(int precision, int kc, int64_t cap);

struct SobolevCall {
    const FaceData* fd = nullptr;
    PairPlan plan;
    int precision = 0;
    double s = 0.0;            // A's kernel is |d|^-2s (order 2s)
    const double* V = nullptr; // nV x 3, FP64
    const int32_t* F = nullptr;
    int64_t nV = 0, nF = 0;
    const int32_t* vf_off = nullptr;   // faces around each vertex (3 * face + corner)
    const int32_t* vf_idx = nullptr;
    void* fu = nullptr;        // sobolev_face_bytes()
    double* part = nullptr;    // [n_split][4 kc][irows]
    double* z = nullptr;       // [4 kc][irows]
    // symmetric pair kernel (FP32 precisions): its partial buffer, sym_part_floats(nF, 4 kc,
    // sym_band) floats, and the band height in blocks; null for the row-by-row kernel
    float* symp = nullptr;
    int sym_band = 0;
};

// dinv[v] = 1 / (approximate diagonal of A at vertex v), FP32 hi/lo pair terms (c.plan
// that of a one-column FP32 call; c.part and c.z sized for it).  The diagonal leaves out the pairs of faces
// that both contain the vertex.
hipError_t launch_sobolev_diag(const SobolevCall& c, double* dinv, hipStream_t s);

// Columns [c0, c0 + kc) of u (row stride ldu) -> the same columns of Au (row stride ldo),
// kc <= kSobCols.  The pair kernel alone is bracketed by (ev0, ev1) when they are non-null
// (with the symmetric kernel in several bands: the band launches and their reductions).
hipError_t launch_sobolev(const SobolevCall& c, const double* u, int ldu, int kc, double* Au, int ldo,
                          int c0, hipEvent_t ev0, hipEvent_t ev1, hipStream_t s);

// ------------------------------------------------------------------ Krylov vectors
//
// Blocks of vectors Vb[i] = Vb + i * vstride, each n x k row-major.  Reductions are
// deterministic: fixed row chunks per workgroup, partials summed in order.

// Doubles of scratch for krylov_dots with nvec * k <= m outputs.
size_t krylov_scratch_doubles(int m);
// out[i * k + c] = sum_v Vb[i][v, c] * w[v, c] for i < nvec (device out).
hipError_t krylov_dots(const double* Vb, int64_t vstride, int nvec, const double* w, int64_t n, int k,
                       double* scratch, double* out, hipStream_t s);
// w[v, c] -= sum_{i < nvec} h[i * k + c] Vb[i][v, c]  (h on the device).
hipError_t krylov_subtract(double* w, const double* Vb, int64_t vstride, int nvec, const double* h, int64_t n,
                           int k, hipStream_t s);
// x[v, c] = (accumulate ? x[v, c] : 0) + sum_{i < nvec} y[i * k + c] Zb[i][v, c]  (y on the device).
hipError_t krylov_combine(double* x, const double* Zb, int64_t vstride, int nvec, const double* y, int64_t n,
                          int k, bool accumulate, hipStream_t s);
// dst[v, c] = src[v, c] * scale[c]  (scale on the device).
hipError_t krylov_scale(double* dst, const double* src, const double* scale, int64_t n, int k, hipStream_t s);

// Z[v, c] += omega * dinv[v] * V[v, c].
hipError_t krylov_diag_add(double* Z, const double* V, const double* dinv, double omega, int64_t n, int k,
                           hipStream_t s);
// out[l][v, c] = (label[v] == l) for l < nl, c < width: nl blocks of n x width.
hipError_t krylov_indicators(const int32_t* label, int64_t n, int nl, int width, double* out, hipStream_t s);

}  // namespace tp
