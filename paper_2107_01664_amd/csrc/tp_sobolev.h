// The inner-product operator A = B + B0 (Sec. 2.3; discrete terms in Sec. 3.3) applied in
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
};

// Columns [c0, c0 + kc) of u (row stride ldu) -> the same columns of Au (row stride ldo),
// kc <= kSobCols.  The pair kernel alone is bracketed by (ev0, ev1) when they are non-null.
hipError_t launch_sobolev(const SobolevCall& c, const double* u, int ldu, int kc, double* Au, int ldo,
                          int c0, hipEvent_t ev0, hipEvent_t ev1, hipStream_t s);

}  // namespace tp
