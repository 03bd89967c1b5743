// Internal declarations shared by the tpsurf HIP sources (not part of the C-ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "tpsurf.h"

namespace tp {

// ------------------------------------------------------------------ constants

constexpr int kBlock = 256;        // threads per workgroup of the pair kernels
constexpr int kTileJ = 128;        // T faces staged in LDS per tile
constexpr int kMaxCols = 64;       // largest k accepted by the column-batched calls
constexpr int kMaxGroupCols = 9;   // columns handled by one pair / CG kernel instance
constexpr int kMaxComponents = 4096;

// Kinds for the kernel timing statistics.
enum PairKind { kKindEnergy = 0, kKindGrad = 1, kKindFrac = 2 };

// Error flags written by device kernels (one int per condition, plain stores of 1).
enum DevFlag { kFlagBadIndex = 0, kFlagDegenerate = 1, kFlagNonFinite = 2, kFlagCgAbort = 3,
               kNumFlags = 4 };

// ------------------------------------------------------------------ error helpers

void set_error(const std::string& msg);
const char* get_error();

#define TP_HIP(call)                                                                   \
    do {                                                                               \
        hipError_t e_ = (call);                                                        \
        if (e_ != hipSuccess) {                                                        \
            ::tp::set_error(std::string(#call) + ": " + hipGetErrorString(e_));        \
            return TP_E_DEVICE;                                                        \
        }                                                                              \
    } while (0)

#define TP_TRY(expr)                                                                   \
    do {                                                                               \
        tp_status s_ = (expr);                                                         \
        if (s_ != TP_OK) return s_;                                                    \
    } while (0)

// ------------------------------------------------------------------ device info

struct DeviceInfo {
    int device = -1;
    int num_cu = 0;
    int max_threads_per_cu = 0;
};
const DeviceInfo& device_info();

// ------------------------------------------------------------------ face data

// Face quantities for the pair kernels.  Arrays hold `cap` entries; entries past nF are
// padding faces placed far away with zero area and zero normal, so every tile is full.
struct FaceData {
    int64_t nF = 0, cap = 0;
    float4* fx = nullptr;    // (Xhi.x, Xhi.y, Xhi.z, a)  FP32
    float4* fl = nullptr;    // (Xlo.x, Xlo.y, Xlo.z, 0)  FP32, Xlo = X - Xhi rounded
    float4* fn = nullptr;    // (N.x, N.y, N.z, 0)        FP32
    double4* dx = nullptr;   // (X.x, X.y, X.z, a)        FP64
    double4* dn = nullptr;   // (N.x, N.y, N.z, 0)        FP64
    float4* tbox = nullptr;  // per kTileJ faces: (lo, hi) boxes of the FP32 barycenters of the
                             // real faces (2 entries per tile; empty box for padding tiles)
};

// Pair-kernel launch geometry for one problem size.
struct PairPlan {
    int ni = 2;              // i faces per thread
    int n_itiles = 0;        // workgroups along i
    int ntiles_j = 0;        // LDS tiles along j (cap / kTileJ)
    int tiles_per_split = 0;
    int n_split = 0;         // workgroups along j
    int64_t irows = 0;       // n_itiles * kBlock * ni (row stride of the partial buffers)
};

// ------------------------------------------------------------------ kernels (launchers)

// Face geometry from vertices and faces (FP64), written in FP32 hi/lo and FP64 forms.
hipError_t launch_face_geom(const double* V, int64_t nV, const int32_t* F, int64_t nF,
                            const FaceData& fd, int* flags, hipStream_t s);
// Face data from caller-given face quantities (X, N row-major nF x 3, a nF).
hipError_t launch_face_from_quantities(const double* X, const double* N, const double* a,
                                       int64_t nF, const FaceData& fd, int* flags, hipStream_t s);

int64_t face_capacity(int64_t nF, int ni_max);
PairPlan plan_pairs(int64_t nF, int64_t cap, int ni, int occupancy_per_cu);

// Uniform cell grid of the FP64 near field (TP_PREC_FP32_NEAR64), built per geometry on
// the FP32 barycenters (hi parts): g cells per axis on the cube [lo, lo + g / inv_cs)^3,
// cells at least 1.01 x the near radius wide, so the two faces of a near pair lie in the
// same or in adjacent cells.
struct NearGridParams {
    float lo[3];
    float inv_cs;     // cells per unit length
    int g;            // cells per axis
    int n;            // faces in the grid (the real faces of the problem)
};

// One problem's share of an all-pairs launch.  A launch covers up to kMaxPairJobs
// problems of the same precision and exponents; problem m owns the workgroups
// [block0, block0 + n_itiles * n_split) of a 1-D grid, laid out i-tile fastest.  The
// arithmetic of a problem does not depend on the other problems of its launch.
struct PairJob {
    const float4* fx = nullptr;
    const float4* fl = nullptr;
    const float4* fn = nullptr;
    const double4* dx = nullptr;
    const double4* dn = nullptr;
    const void* ub = nullptr;       // face-averaged columns (fractional apply only)
    double* part = nullptr;         // partial buffer [n_split][nacc][irows]
    int64_t irows = 0;
    int n_itiles = 0, tiles_per_split = 0, ntiles_j = 0, block0 = 0;
    float rho2 = 0.f;               // TP_PREC_FP32_NEAR64: pairs with r2 < rho2 are left out
    const float4* tbox = nullptr;   // tile boxes (FaceData::tbox)
    // near-field grid (NearGrid): faces in cell order, their FP32 hi / lo barycenters in
    // that order, [begin, end) of every cell, parameters
    const int32_t* nord = nullptr;
    const float4* nfx = nullptr;
    const float4* nfl = nullptr;
    const int2* ncell = nullptr;
    const NearGridParams* ngp = nullptr;
};
constexpr int kMaxPairJobs = 16;
PairJob make_pair_job(const FaceData& fd, const PairPlan& pl, double* part, const void* ub = nullptr);

// All-pairs kernels over njobs problems (any njobs >= 1; launched in chunks of
// kMaxPairJobs).  Partial buffers are [n_split][nacc][irows] doubles.
hipError_t launch_pairs_energy(const PairJob* jobs, int njobs, int precision, double alpha,
                               double beta, hipStream_t s);
hipError_t launch_pairs_grad(const PairJob* jobs, int njobs, int precision, double alpha,
                             double beta, hipStream_t s);
// ub: face-averaged columns, FP32 [cap][kp] (kp = k rounded up to 4) or FP64 [cap][kp].
hipError_t launch_pairs_frac(const PairJob* jobs, int njobs, int precision, double sigma, int k,
                             hipStream_t s);
PairPlan plan_for(int kind, int precision, int k, int64_t nF, int64_t cap);

// Symmetric all-pairs kernels (each unordered pair once, both rows; FP32 pair terms).  Faces
// are cut into nB blocks of frac_sym_block_faces(); a launch takes the pairs of blocks (a, b),
// b >= a, of a band of rows a in [a0, a1), and writes, per face and slice, kc FP32 partial
// sums: row T's sums of pair (a, b) to partT[a - a0][c][T] ([K][kc][ldp]) and row S's to
// partS[b][c][S - a0 blk] ([nB][kc][K blk]), K = a1 - a0 at most the band height the buffer
// was sized for.  With a single band (K = nB) the two regions are one array [nB][kc][ldp].
// launch_reduce_sym_band then adds the band's slices to out[c * out_stride + i] in FP64, in
// the slice order of a single launch (rows a < block of i, then b >= block of i, then the
// near field extra), so the result does not depend on the band height.
struct SymFracArgs {
    const float4* fx = nullptr;
    const float4* fl = nullptr;
    const float* ub = nullptr;
    const float4* tbox = nullptr;
    float* part = nullptr;    // row T's sums: [K][kc][ldp]
    float* partS = nullptr;   // row S's sums: [nB][kc][ldS]
    int64_t ldp = 0;          // nB * frac_sym_block_faces()
    int64_t ldS = 0;          // K * frac_sym_block_faces() (ldp with a single band)
    int nB = 0;               // blocks of frac_sym_block_faces() faces holding the real faces
    int a0 = 0, a1 = 0;       // band of rows
};
int frac_sym_block_faces();
// Band height (blocks) whose partial buffer stays within max_bytes (nB when a single band
// fits, else at least 1), and the FP32 entries of that buffer.
int sym_band_blocks(int64_t nF, int kc, double max_bytes);
size_t sym_part_floats(int64_t nF, int kc, int K);
// Unordered pairs of blocks (a, b), b >= a, with a in [a0, a1).
int64_t sym_band_units(int64_t nF, int a0, int a1);
// Pointers and leading dimensions of the two slice regions of a buffer for band height K.
void sym_regions(float* part, int64_t nF, int kc, int K, float*& partT, float*& partS, int64_t& ldp, int64_t& ldS);
// The pair kernel for rows [a0, a1) of bands of height K (kc = 1..9 columns; precision as for
// the row-owned kernel, not TP_PREC_FP64).
hipError_t launch_frac_sym(const FaceData& fd, const float* ub, float* part, int K, int a0, int a1, int precision,
                           double sigma, int kc, hipStream_t s);
hipError_t launch_reduce_sym_band(const float* part, int64_t nF, int kc, int K, int a0, int a1, const double* extra,
                                  double* out, int64_t out_stride, hipStream_t s);
// Symmetric E + dE: the seven outputs per face and slice (kc = 7 above); with
// TP_PREC_FP32_NEAR64 pairs closer than sqrt(rho2) are left to the near field.
hipError_t launch_grad_sym(const FaceData& fd, float* part, int K, int a0, int a1, int precision, double alpha,
                           double beta, float rho2, hipStream_t s);

// Symmetric energy (each unordered pair once; FP32 pair terms): one FP64 partial per pair of
// blocks, sym_units(nF) of them, into upart (their sum, plus the near field's
// sum_i a_i near[i] when pairs closer than sqrt(rho2) are left to it, is E).
int64_t sym_units(int64_t nF);
hipError_t launch_energy_sym(const FaceData& fd, double* upart, int precision, double alpha, double beta, float rho2,
                             hipStream_t s);
hipError_t launch_area_times(const FaceData& fd, const double* near, int64_t n, double* out, hipStream_t s);

// Sum the n_split partials of every accumulator in split order: out[acc][i].
hipError_t launch_reduce_splits(const double* part, int n_split, int nacc, int64_t irows,
                                int64_t n, double* out, int64_t out_stride, hipStream_t s);

// Mesh / sparse kernels.
hipError_t launch_check_indices(const int32_t* F, int64_t nF, int64_t nV, int* flags, hipStream_t s);
hipError_t launch_vf_count(const int32_t* F, int64_t nF, int64_t nV, int32_t* deg, hipStream_t s);
hipError_t launch_scan(const int32_t* in, int64_t n, int32_t* out_excl /* n + 1 */, hipStream_t s);
hipError_t launch_vf_fill(const int32_t* F, int64_t nF, int64_t nV, const int32_t* off,
                          int32_t* cursor, int32_t* idx, hipStream_t s);
hipError_t launch_sort_rows(const int32_t* off, int64_t n, int32_t* idx, hipStream_t s);
hipError_t launch_lap_pattern_count(const int32_t* F, int64_t nV, const int32_t* vf_off,
                                    const int32_t* vf_idx, int32_t* cand, int32_t* cnt,
                                    hipStream_t s);
hipError_t launch_lap_pattern_fill(int64_t nV, const int32_t* vf_off, const int32_t* cand,
                                   const int32_t* lap_off, int32_t* lap_col, hipStream_t s);
hipError_t launch_cotan_values(const double* V, const int32_t* F, int64_t nV,
                               const int32_t* vf_off, const int32_t* vf_idx,
                               const int32_t* lap_off, const int32_t* lap_col, double* lap_val,
                               hipStream_t s);
hipError_t launch_grad_gather(const double* V, const int32_t* F, int64_t nV, int64_t nF,
                              const int32_t* vf_off, const int32_t* vf_idx,
                              const double* gface, int64_t gstride, double* dE, hipStream_t s);
// ubar of columns u[:, 0..k) (row stride ldu) into ub [cap][kp].
hipError_t launch_face_avg(const int32_t* F, int64_t nF, int64_t cap, const double* u, int ldu,
                           int k, int kp, int precision, void* ub, hipStream_t s);
hipError_t launch_ut_gather(const int32_t* F, int64_t nV, const int32_t* vf_off,
                            const int32_t* vf_idx, const FaceData& fd, const double* z,
                            int64_t zstride, int k, int kout, int c0, double* Lu, hipStream_t s);
hipError_t launch_volume_gradient(const double* V, const int32_t* F, int64_t nV,
                                  const int32_t* vf_off, const int32_t* vf_idx, double* out,
                                  int ldo, int c0, hipStream_t s);
hipError_t launch_face_volume(const double* V, const int32_t* F, int64_t nF, double* vol6,
                              hipStream_t s);
hipError_t launch_spmm(int64_t n, const int32_t* off, const int32_t* col, const double* val,
                       const double* x, int ldx, int k, double* y, int ldy, hipStream_t s);

// Deterministic reductions.  `scratch` must hold reduce_scratch_doubles() doubles.
size_t reduce_scratch_doubles(int ncols);
// out[c] = sum_i x[i*ldx + c] * (y ? y[i*ldy + c] : 1) for c < ncols, written to device out.
hipError_t launch_dot_cols(const double* x, int ldx, const double* y, int ldy, int64_t n,
                           int ncols, double* scratch, double* out, hipStream_t s);
// out = max_i |x_i| over n rows of 3 (Euclidean row norms), device scalar.
hipError_t launch_max_rownorm3(const double* x, int64_t n, double* scratch, double* out,
                               hipStream_t s);
// Per-component means of k columns, then x -= mean[comp].
hipError_t launch_project_mean(double* x, int ldx, int k, int64_t n, const int32_t* comp,
                               const double* inv_count, int ncomp, double* scratch,
                               hipStream_t s);
size_t project_scratch_doubles(int k, int ncomp);
// Vertex pins: the solver's copy of the cotan values with the pinned rows and columns
// replaced by the identity; zeroing of the pinned rows of k columns.
hipError_t launch_pin_values(int64_t n, const int32_t* off, const int32_t* col, const double* val,
                             const int8_t* pinned, double* out, hipStream_t s);
hipError_t launch_zero_pinned(double* x, int ldx, int k, int64_t n, const int8_t* pinned, hipStream_t s);

// y = a*x + b*y style updates on n x 3 blocks: out = x + sum_m coef[m] * Y[:, cols_m].
hipError_t launch_axpy_block3(int64_t n, const double* x, int ldx, double a,
                              const double* Y, int ldy, int ncoef, const double* coef_host,
                              const int* cols_host, double* out, int ldo, hipStream_t s);
hipError_t launch_copy_cols(int64_t n, const double* x, int ldx, int k, double* y, int ldy,
                            hipStream_t s);

// Barnes-Hut approximation (tp_bh.hip).  Buffers are owned by the problem.
struct BhBuffers {
    double* flo = nullptr;        // [nF][3] face boxes
    double* fhi = nullptr;
    double* fr2 = nullptr;        // [nF]
    double* box = nullptr;        // [6] barycenter bounding box
    uint64_t* keys_in = nullptr;  // [nF]
    uint64_t* keys_out = nullptr; // [nF]
    void* sort_tmp = nullptr;
    size_t sort_bytes = 0;
    int32_t* order = nullptr;     // [nF] sorted position -> face
    int32_t* pos = nullptr;       // [nF] face -> sorted position
    double* na = nullptr;         // [M]  (M = 2P nodes, heap order)
    double* nsx = nullptr;        // [M][3]
    double* nX = nullptr;         // [M][3]
    double* nlo = nullptr;        // [M][3]
    double* nhi = nullptr;        // [M][3]
    double* nr2 = nullptr;        // [M]
    double* gS = nullptr;         // [7][nF]
    double* eS = nullptr;         // [nF]
    double* accF = nullptr;       // [4][nF]
    double* accN = nullptr;       // [4][M]
    unsigned long long* counts = nullptr;   // [2] far, near terms
};
size_t bh_node_count(int64_t nF, int leaf, int64_t* P_out);
size_t bh_sort_temp_bytes(int64_t nF);
// Faces sorted by (Morton code of the barycenter, orig[face] or the face index when orig is
// NULL): sorted internal indices into b.order (uses b.box, b.keys_*, b.pos, b.sort_tmp).
hipError_t launch_morton_order(const BhBuffers& b, const FaceData& fd, int64_t nF, const int32_t* orig,
                               hipStream_t s);
// Tree of the faces described by fd, whose vertices are V; orig = the caller's face numbers.
hipError_t launch_bh_build(const BhBuffers& b, const double* V, const int32_t* F, const int32_t* orig, int64_t nF,
                           int leaf, const FaceData& fd, hipStream_t s);
// E_BH rows into b.eS and, with grad, the per-face partial derivatives into gface
// ([7][gstride]: dE/dX, dE/dN, dE/da).
hipError_t launch_bh_eval(const BhBuffers& b, int64_t nF, int leaf, double theta, int precision, double alpha,
                          double beta, const FaceData& fd, bool grad, double* gface, int64_t gstride,
                          hipStream_t s);
// L^sigma's kernel sums with Barnes-Hut (theta > 0) on the built tree: face averages ub
// ([cap][kp], kp = k rounded up to 4, zero padded; FP64 for TP_PREC_FP64 else FP32), node
// moments nm ([2P][kp] doubles), output z(S) (the row sums without a_S) at z[c * zstride + S],
// k <= kMaxGroupCols.
// Block cluster tree of the fractional operator's kernel matrix (device CSR lists): per row
// node the admissible column nodes, per row leaf the inadmissible column leaves.
struct BctLists {
    const int32_t* far_off = nullptr;    // [2P + 1]
    const int32_t* far_col = nullptr;
    const int32_t* near_off = nullptr;   // [P + 1] (leaf index = node - P)
    const int32_t* near_col = nullptr;   // leaf indices
};
// L^sigma's kernel sums by hierarchical multiplication on the lists; nm [2P][kp] node moments,
// yt [2P][kp + 4] far-field values, output as launch_bh_frac.
hipError_t launch_bct_frac(const BhBuffers& b, const BctLists& bl, int64_t nF, int leaf, int precision,
                           double sigma, const FaceData& fd, const void* ub, int kp, int k, double* nm, double* yt,
                           double* z, int64_t zstride, hipStream_t s);
hipError_t launch_bh_frac(const BhBuffers& b, int64_t nF, int leaf, double theta, int precision, double sigma,
                          const FaceData& fd, const void* ub, int kp, int k, double* nm, double* z, int64_t zstride,
                          hipStream_t s);

// Buffers of the near-field grid of one problem (device memory owned by the problem).
struct NearGrid {
    uint32_t* kin = nullptr;      // [nF] cell index of each face
    uint32_t* kout = nullptr;     // [nF] sorted
    int32_t* vin = nullptr;       // [nF] face numbers
    int32_t* vout = nullptr;      // [nF] faces in cell order (ties in face order)
    float4* sfx = nullptr;        // [nF] fx in cell order
    float4* sfl = nullptr;        // [nF] fl in cell order
    int2* cell = nullptr;         // [gmax^3] (begin, end) in cell order; empty cells (0, 0)
    void* sort_tmp = nullptr;
    size_t sort_bytes = 0;
    int gmax = 1;
    NearGridParams* prm = nullptr;
};
int near_grid_gmax(int64_t nF);                 // cells per axis at most: cbrt(8 nF), 1..128
size_t near_grid_sort_temp_bytes(int64_t nF);
// Grid of the first nF faces of fd for the squared near radius rho2.
hipError_t launch_near_grid_build(const NearGrid& g, const FaceData& fd, int64_t nF, float rho2, hipStream_t s);

// FP64 near field (TP_PREC_FP32_NEAR64), as one launch over the problems of a batch: for
// every face S, the pairs (S, T), T != S, whose FP32 hi+lo squared barycenter distance is
// below the job's rho2 (exactly the pairs the FP32 kernels leave out), summed in FP64 into
// the job's partial slice ([7][irows] with grad, else [irows]).  The candidates T of S are
// the faces of the 27 grid cells around S's cell.
hipError_t launch_near64(const PairJob* jobs, int njobs, double alpha, double beta, bool grad, hipStream_t s);
int near_block_faces();           // faces S per near-field workgroup (n_itiles of a near job)

}  // namespace tp
