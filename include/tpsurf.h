/*
 * tpsurf.h -- C-ABI of the tangent-point hot path of "Repulsive Surfaces"
 * (Yu, Brakensiek, Schumacher, Crane, ACM TOG 2021) on AMD MI355X (gfx950).
 *
 * What the library computes, on a closed triangle mesh M = (V, F) with embedding f:
 *   - the discrete tangent-point energy E (Sec. 3.1, eq. DiscreteEnergy with the kernel
 *     of eq. DiscreteTangentPointKernel), with independent exponents (alpha, beta),
 *     the paper's choice being (p, 2p) with p = 6 (Sec. 2.1);
 *   - its differential dE with respect to the vertex positions (Sec. 3.1, chain rule);
 *   - the forward application of the fractional operator L^sigma (Sec. 2.4, eq.
 *     DiscreteLaplacianQuartic) in the factored kernel-matrix form of Sec. 5.1.1 / App. A;
 *   - the preconditioner A~^{-1} = C^{-1} L^sigma C^{-1} of Sec. 5.2, with both Poisson
 *     solves done by FP64 conjugate gradients on the cotan stiffness matrix C;
 *   - one projected descent step with total-area and total-volume constraints (Sec. 3,
 *     eq. SaddleProblem via the Schur complement of Sec. 5.3, Armijo line search, and the
 *     corrective projection of Sec. 5.3.1), A~^{-1} standing in for A_3^{-1}.
 *
 * Conventions shared by every entry point
 *   - V: vertex positions, nV x 3, row-major double.  F: faces, nF x 3, row-major int32,
 *     0-based vertex indices, consistently oriented (orientation only fixes the sign of
 *     the volume; the energy uses the normal projector, which ignores it).
 *   - Unless stated otherwise, array arguments are DEVICE pointers on the current HIP
 *     device (for example torch tensors' data_ptr()), scalars out-parameters are HOST
 *     pointers.  The caller owns every buffer; the library keeps no pointer to caller
 *     memory after a call returns.
 *   - `stream` is a hipStream_t passed as void* (NULL = the default stream).  Every call
 *     is ordered on that stream and returns after its work has completed.
 *   - Errors are returned as tp_status; no exception crosses the ABI.  tp_last_error()
 *     gives a message for the calling thread.  On error the outputs are undefined, except
 *     for TP_E_NOT_CONVERGED, where outputs and reports are written.
 *   - Results are deterministic (fixed reduction orders, no floating-point atomics), with
 *     one exception: the Barnes-Hut differential (theta > 0) adds its target-side terms
 *     with floating-point atomics, so its last bits can differ from run to run.
 */
#ifndef TPSURF_H
#define TPSURF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TPSURF_VERSION 1

#if defined(__GNUC__) || defined(__clang__)
#define TP_API __attribute__((visibility("default")))
#else
#define TP_API
#endif

typedef enum {
    TP_OK = 0,
    TP_E_INVALID_ARGUMENT = 1,       /* bad size, pointer, exponent or option           */
    TP_E_DEGENERATE_FACE = 2,        /* a face has zero area: its normal is undefined  */
    TP_E_BAD_INDEX = 3,              /* a face refers to a vertex outside [0, nV)      */
    TP_E_NONFINITE = 4,              /* non-finite input or result (e.g. two faces with
                                        coincident barycenters make the kernel infinite) */
    TP_E_NOT_CONVERGED = 5,          /* CG reached cg_maxiter before cg_rtol            */
    TP_E_OUT_OF_MEMORY = 6,
    TP_E_SINGULAR_CONSTRAINTS = 7,   /* the Schur matrix J A~^{-1} J^T is singular      */
    TP_E_DEVICE = 8                  /* a HIP runtime error                             */
} tp_status;

/* Arithmetic of the all-pairs sums.  The terms of each 128-face tile are summed in FP32
 * (FP64 for TP_PREC_FP64) and the per-face running sums are FP64, except in the two
 * precision-sweep modes 4 and 5. */
typedef enum {
    TP_PREC_FP32_HILO = 0,  /* FP32 pair terms; barycenter differences from hi+lo FP32
                               splits of the FP64 barycenters                             */
    TP_PREC_FP32 = 1,       /* FP32 pair terms from FP32-rounded barycenters              */
    TP_PREC_FP64 = 2,       /* FP64 pair terms                                            */
    TP_PREC_FP32_NEAR64 = 3, /* as TP_PREC_FP32_HILO for the energy and its differential,
                               except that pairs whose barycenters are closer than twice
                               the mean edge length of the problem's first mesh (tested on
                               the FP32 hi+lo distance) are summed in FP64; the fractional
                               apply is as TP_PREC_FP32_HILO (default)                     */
    TP_PREC_FP32_ACC32 = 4, /* as TP_PREC_FP32, with each face's running sum of E and dE
                               terms over its j-split kept in FP32 (plain additions); the
                               sums over splits, the chain rule and the total stay FP64.
                               For precision studies only                                  */
    TP_PREC_FP32_KAHAN = 5  /* as TP_PREC_FP32_ACC32 with Kahan's compensated summation of
                               the per-face running sums. For precision studies only      */
} tp_precision;

typedef struct {
    double alpha;        /* numerator exponent, default 6 (p, Sec. 2.1); must be > 1    */
    double beta;         /* denominator exponent, default 12 (2p); must be > 0          */
    double sigma;        /* order parameter of L^sigma; < 0 selects 2 - s with
                            s = (beta - 2)/alpha (= 2 - 2/p when beta = 2 alpha,
                            Sec. 2.3 and Sec. 5.2); default -1 -> 1/3 at p = 6           */
    int    precision;    /* tp_precision, default TP_PREC_FP32_NEAR64                    */
    double cg_rtol;      /* CG stops when ||b - C x|| <= cg_rtol ||b||, default 1e-10   */
    int    cg_maxiter;   /* default 20000                                               */
    int    cg_precond;   /* 1: two-level additive Schwarz preconditioner (default, used
                            when the mesh has at most 256 blocks of 128 vertices);
                            0: unpreconditioned CG                                        */
    double theta;        /* 0 (default): E and dE by the direct all-pairs sums; > 0: the
                            Barnes-Hut approximation of Sec. 4 with opening parameter
                            theta (the paper's default is 0.5), see tp_problem_bh_stats  */
    int    leaf_size;    /* faces per Barnes-Hut leaf, 1..64, default 8 (Sec. 4.1)       */
    double chi;          /* 0 (default): the fractional operator's kernel sums directly
                            (or by Barnes-Hut when theta > 0); > 0: by the block cluster
                            tree and hierarchical multiplication of Sec. 5.1.4-5.1.5 with
                            separation parameter chi (the paper's default is 0.5) on the
                            Barnes-Hut tree: node pairs with max(r_I, r_J) < chi
                            dist(box_I, box_J) are rank-one blocks k(X_I, X_J), leaf pairs
                            that are not separated are exact (App. B: upward pass of node
                            sums, far-field products per node, downward pass to faces);
                            see tp_problem_bct_stats                                     */
    int    sym_pairs;     /* direct FP32 sums of E, E + dE, the fractional apply and the
                            operator A = B + B0: -1 (default) symmetric from 16,384 faces
                            on, 0 row by row (every ordered pair evaluated for its row), 1
                            symmetric at any size; symmetric means every unordered pair
                            evaluated once for both rows (the kernel values K(S,T) and
                            K(T,S), |d|^-(2 sigma + 2) and |d|^-2s come from the same d);
                            E and E + dE stay row by row in precisions 4 and 5            */
    int    sym_band;      /* the symmetric kernels take the rows of 256-face blocks in bands,
                            one launch and one FP64 reduction per band, so that their FP32
                            partial buffer (2 * band * k * nF floats, or ceil(nF/256) * k *
                            nF with one band) stays within 512 MB; 0 (default): the tallest
                            such band; > 0: at most that many blocks per band.  The sums
                            are added in the same order for every band height, so results
                            do not depend on it                                            */
} tp_params;

/* Fill *p with the defaults above. */
TP_API tp_status tp_params_default(tp_params* p);

/* ---------------------------------------------------------------- stateless calls */

/* E = sum_S sum_{T != S} K(S,T) a_S a_T (eq. DiscreteEnergy; the diagonal is excluded).
 * E_out: host pointer to one double. */
TP_API tp_status tp_energy(const double* V, int64_t nV, const int32_t* F, int64_t nF,
                    const tp_params* params, double* E_out, void* stream);

/* E and dE (Sec. 3.1).  dE_out: device, nV x 3 row-major double. */
TP_API tp_status tp_gradient(const double* V, int64_t nV, const int32_t* F, int64_t nF,
                      const tp_params* params, double* E_out, double* dE_out, void* stream);

/* E on face quantities directly: X, N nF x 3 row-major double (N unit), a nF double,
 * all device pointers.  E depends on the mesh only through these (Sec. 4.1 writes the
 * kernel as K_p(X_S, P_S; X_T)). */
TP_API tp_status tp_energy_faces(const double* X, const double* N, const double* a, int64_t nF,
                          const tp_params* params, double* E_out, void* stream);

/* tp_energy_faces without any allocation, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).
 * Same arguments, kernels and result as tp_energy_faces (partial sums may be split
 * differently, so the last bits can differ).  All device scratch lives in one static
 * device array of 32 MiB that each GPU the library runs on holds until the process ends;
 * nF is limited to 2 <= nF <= 65536 (TP_E_INVALID_ARGUMENT above that, before any device
 * work).  theta > 0 and TP_PREC_FP32_NEAR64 are rejected as in tp_energy_faces.  Every
 * call on a GPU shares that GPU's array: calls that overlap on one GPU (other streams or
 * threads) race and must be serialised by the caller.  The call returns after the result
 * has been copied to E_out (a stream synchronisation). */
TP_API tp_status tp_energy_faces_noalloc(const double* X, const double* N, const double* a, int64_t nF,
                                  const tp_params* params, double* E_out, void* stream);

/* Lu = L^sigma u for k columns (eq. DiscreteLaplacianQuartic, factored as
 * 2 U^T [diag(diag(a)^-1 H a) - H] U of Sec. 5.1.1, H_ST = (1 - delta_ST)|X_S - X_T|^-(2 sigma + 2)).
 * u, Lu_out: device, nV x k row-major double, 1 <= k <= 64. */
TP_API tp_status tp_fractional_apply(const double* V, int64_t nV, const int32_t* F, int64_t nF,
                              const tp_params* params, const double* u, int k,
                              double* Lu_out, void* stream);

/* Au = A u = (B + B0) u for k columns: the operator of the paper's inner product (Sec. 2.4,
 * high- and low-order terms; discrete forms eqs. DiscreteHighOrderTerm and
 * DiscreteLowOrderTerm of Sec. 3.2.1), applied in the factored form of Sec. 5.1.2 / 5.1.3:
 *   B u  = 2 (diag(a) D)^T [diag(diag(a)^-1 H a) - H] diag(a) D u,  H_ST = (1 - delta_ST)|X_S - X_T|^-2s,
 *   B0 u = 2 U^T [diag(diag(a)^-1 H0 a) - H0] U u,  H0_ST = H_ST (K2(S,T) + K2(T,S)) / 2,
 * with s = (beta - 2) / alpha (sigma = s - 1 in the paper's notation for these terms),
 * K2(S,T) = (N_S . (X_S - X_T))^2 / |X_S - X_T|^4, D u(S) the gradient of the piecewise
 * linear u on face S (N_S x opposite edge / (2 a_S) per corner) and U the face average times
 * the area.  A annihilates constants; it is symmetric positive semidefinite.  Each column is
 * one scalar function; the operator A_3 of the descent direction applies A to the three
 * coordinate columns.  u, Au_out: device, nV x k row-major double, 1 <= k <= 64; the caller
 * owns both.  The pair terms follow params->precision (FP64, or FP32 with FP64 sums; the
 * near-field FP64 option of the energy applies FP32 hi/lo here).  Errors: TP_E_INVALID_ARGUMENT
 * for NULL pointers or k outside [1, 64], and the mesh checks of tp_problem_create. */
TP_API tp_status tp_sobolev_apply(const double* V, int64_t nV, const int32_t* F, int64_t nF,
                                  const tp_params* params, const double* u, int k,
                                  double* Au_out, void* stream);

/* Report of one preconditioner application (two CG solves). */
typedef struct {
    int    cg_iters[2];      /* largest iteration count over the columns, per solve      */
    double cg_relres[2];     /* largest final ||r||/||b|| over the columns, per solve     */
    double t_ms[4];          /* CG 1, fractional apply, CG 2, total (device time)        */
} tp_solve_report;

/* x = A~^{-1} b = C^+ P L^sigma C^+ P b columnwise (Sec. 5.2): P subtracts the unweighted
 * per-connected-component mean, C^+ P y is the per-component mean-zero solution of
 * C x = P y by FP64 CG.  b, x_out: device, nV x k row-major, 1 <= k <= 64.
 * report may be NULL. */
TP_API tp_status tp_precond_apply(const double* V, int64_t nV, const int32_t* F, int64_t nF,
                           const tp_params* params, const double* b, int k, double* x_out,
                           tp_solve_report* report, void* stream);

/* ----------------------------------------------------- resident problem (stateful) */

/* A problem keeps the topology (vertex-face incidence, cotan sparsity, components), the
 * current vertex positions and all work buffers on the device, so repeated calls do no
 * allocation or host-side preprocessing.  A problem is used by one thread at a time. */
typedef struct tp_problem tp_problem;

/* Copies V and F (device pointers) into a new problem on the current device. */
TP_API tp_status tp_problem_create(const double* V, int64_t nV, const int32_t* F, int64_t nF,
                            const tp_params* params, void* stream, tp_problem** out);
TP_API void      tp_problem_destroy(tp_problem* prob);

/* Replace / read the current vertex positions (device, nV x 3).
 * When the previous positions were used by a Poisson solve, set_vertices also starts the
 * cotan values, the solvers' matrix and the preconditioner's set-up for the new positions
 * on a second stream of the problem (default priority), after the work enqueued so far on
 * the problem's stream; tp_precond_step does the same at its start.  The energy, gradient
 * and fractional-apply calls run beside it; every other call on the problem first makes
 * the problem's stream wait for it, and tp_problem_destroy waits for both streams.  Results
 * are the same bit for bit as with the set-up done on the problem's stream. */
TP_API tp_status tp_problem_set_vertices(tp_problem* prob, const double* V);
TP_API tp_status tp_problem_get_vertices(tp_problem* prob, double* V_out);

/* Same operations as the stateless calls, on the problem's current vertices. */
TP_API tp_status tp_problem_energy(tp_problem* prob, double* E_out);
TP_API tp_status tp_problem_gradient(tp_problem* prob, double* E_out, double* dE_out);
TP_API tp_status tp_problem_fractional_apply(tp_problem* prob, const double* u, int k, double* Lu_out);
TP_API tp_status tp_problem_sobolev_apply(tp_problem* prob, const double* u, int k, double* Au_out);

/* Static obstacle (Sec. 7.3.2): a fixed mesh (Vo: nVo x 3 double, Fo: nFo x 3 int32, device,
 * copied at the call) that repels the surface with the potential
 *   E_obs = sum_T a_T sum_{S in obstacle} a_O(S) |X_O(S) - X_T|^-p
 * (the obstacle potential of the paper evaluated at the barycenter of every face T of the
 * surface and integrated over T; FP64).  With params.theta = 0 the sums are direct; with
 * theta > 0 they use Barnes-Hut, as the end of Sec. 7.3.2 suggests: a tree over the
 * obstacle's faces (the tree of the energy's Barnes-Hut, built once at this call), and for
 * the barycenter X_T of each surface face, a point, node I is admissible when
 * r_I^2 < theta^2 dist(X_T, box_I)^2 and then contributes a_I |X_I - X_T|^-p; leaves that
 * are not admissible contribute face by face (see tp_problem_obstacle_stats).  With weight > 0 every
 * later descent step of this problem minimises E + weight E_obs (gradient, line search and
 * the report's energies).  nFo = 0 or weight = 0 removes the obstacle.  Errors:
 * TP_E_INVALID_ARGUMENT for bad sizes, indices, p <= 0 or weight < 0. */
TP_API tp_status tp_problem_set_obstacle(tp_problem* prob, const double* Vo, int64_t nVo, const int32_t* Fo,
                                         int64_t nFo, double p, double weight);

/* Term counts of the last obstacle evaluation: far (node) and near (face) terms summed over
 * the surface's faces; with theta = 0, far = 0 and near = nF x nFo; both 0 without an
 * obstacle. */
TP_API tp_status tp_problem_obstacle_stats(tp_problem* prob, int64_t* far_terms, int64_t* near_terms);
/* E_out = E_obs (unweighted) at the current vertices; dE_out (device nV x 3, or NULL) its
 * differential with respect to the surface's vertex positions. */
TP_API tp_status tp_problem_obstacle_energy(tp_problem* prob, double* E_out, double* dE_out);

/* Vertex pin constraints (Sec. 7.1.2): the vertices idx[0..n) (HOST int32 indices) keep
 * their current positions in every later step.  Following Sec. 7.2 (linear positional
 * rows go into the operator rather than the Schur complement), their rows are appended to
 * both Laplacians of the preconditioner: each Poisson solve (of the step, and of
 * tp_problem_poisson_solve / tp_problem_precond_apply) returns zero at the pinned vertices
 * and solves C x = b on the other rows, and a component holding a pin has no mean-zero
 * projection.  The direction and the corrective step therefore vanish at the pins.  n = 0
 * removes all pins.  TP_E_BAD_INDEX for an index outside [0, nV); a step with pins and
 * barycenter_motion = 1 or solver = 1 is TP_E_INVALID_ARGUMENT. */
TP_API tp_status tp_problem_set_pins(tp_problem* prob, const int32_t* idx, int64_t n);

/* Implicit obstacles and attractors (Sec. 7.3.3) on analytic signed distances d: kind 0 a
 * plane, d(x) = (q . x - c) / |q|; kind 1 a sphere, d(x) = |x - q| - c (c > 0 the radius;
 * q: host pointer to 3 doubles).  Potential weight * d^-p for an obstacle (attract = 0; a
 * face barycenter with d <= 0 makes it +infinity for every p, and the line search rejects
 * such steps; a step whose corrected positions put a barycenter there ends with
 * TP_E_NONFINITE),
 * weight * |d|^p for an attractor (attract = 1), evaluated at the face barycenters and
 * integrated with the face areas, summed over the primitives (at most 8) and added to the
 * objective of every later step.  kind < 0 removes them all.  TP_E_INVALID_ARGUMENT for a
 * bad kind, p <= 0, weight <= 0, a zero plane normal or radius, or a ninth primitive. */
TP_API tp_status tp_problem_add_implicit(tp_problem* prob, int kind, const double* q, double c, double p,
                                         double weight, int attract);
/* E_out = the weighted sum of the implicit potentials at the current vertices; dE_out
 * (device nV x 3, or NULL) its differential. */
TP_API tp_status tp_problem_implicit_energy(tp_problem* prob, double* E_out, double* dE_out);

/* Report of one GMRES solve with A (tp_problem_sobolev_solve). */
typedef struct {
    int    iters;             /* GMRES iterations (one preconditioner and one A product each) */
    int    cycles;            /* restart cycles started                                       */
    double relres;            /* largest |P b - A x| / |P b| over the columns (true residual) */
    int    precond_cg_iters;  /* CG iterations summed over the preconditioner's Poisson solves */
    double t_ms;              /* device time of the whole solve                                */
    double omega;             /* weight of the diagonal term (precond = 1), else 0             */
} tp_gmres_report;

/* x = A^+ P b columnwise, A = B + B0 as in tp_sobolev_apply: the solve of the descent step
 * done with the true operator (Sec. 5.4: an iterative method with the preconditioner
 * of Sec. 5.2 and a zero initial guess; products with A evaluated directly rather than with
 * the block cluster tree).  A annihilates the global constants only: its low-order term
 * couples the connected components.  P subtracts the global mean and x has global mean
 * zero; with 2 to 16 components the preconditioner is completed by an exact coarse solve
 * on the component indicators (their relative translations), with more than 16 P
 * subtracts every component's mean and x solves P A x = P b on that subspace (relative
 * translations left out).  Right-preconditioned GMRES
 * restarted every `restart` iterations, preconditioner A~^{-1} (tp_problem_precond_apply)
 * kept per iteration (flexible form, since it is applied through CG solves); the k columns
 * are independent systems iterated together.  Stops when every column's true residual
 * |P b - A x| / |P b| <= rtol, or after maxiter iterations (TP_E_NOT_CONVERGED; x and the
 * report are written).  With FP32 pair terms the residual is that of the FP32 operator,
 * which is reproducible but not exact: rtol near 1e-7 and below needs TP_PREC_FP64.
 * precond = 0: the preconditioner of Sec. 5.2 alone.  precond = 1: A~^{-1} + omega diag(A)^{-1},
 * an addition to the paper: A~^{-1} under-weights the highest frequencies (its face
 * averages lose them; the eigenvalue spread of A~^{-1} A grows about fourfold per halving
 * of the edge length), which the diagonal of A (without the pairs of faces sharing the
 * vertex) covers; omega = w^T A~^{-1} w / w^T v with w = A v on the coordinate functions.
 * b, x_out: device, nV x k row-major double; b is not modified.  Requires rtol > 0,
 * 1 <= restart <= 100, (restart + 1) k <= 1024, maxiter >= 1, precond 0 or 1
 * (TP_E_INVALID_ARGUMENT).
 * The preconditioner's Poisson solves run to relative residual 1e-3 (or cg_rtol if looser):
 * the flexible form needs no more, since the residual is formed with the directions the
 * preconditioner returned.
 * Device memory: 2 (restart + 1) nV k doubles of Krylov vectors, held by the problem. */
TP_API tp_status tp_problem_sobolev_solve(tp_problem* prob, const double* b, int k, double rtol, int restart,
                                          int maxiter, int precond, double* x_out, tp_gmres_report* report);
TP_API tp_status tp_problem_precond_apply(tp_problem* prob, const double* b, int k, double* x_out,
                                   tp_solve_report* report);

/* x = C^+ P b columnwise: the per-component mean-zero solution of the cotan Poisson
 * problem C x = P b by FP64 CG (one of the two solves inside A~^{-1}, Sec. 5.2).
 * b, x_out: device, nV x k row-major, 1 <= k <= 64.  report (may be NULL) receives the
 * largest iteration count and final true relative residual in cg_iters[0], cg_relres[0]. */
TP_API tp_status tp_problem_poisson_solve(tp_problem* prob, const double* b, int k, double* x_out,
                                          tp_solve_report* report);

/* Options of one descent step. */
typedef struct {
    double tau0;             /* initial step; <= 0 selects the step whose largest vertex
                                move is half the mean edge length of the initial mesh     */
    int    line_search;      /* 1: Armijo backtracking from tau0; 0: take tau0           */
    double armijo_c;         /* sufficient-decrease constant, default 1e-4               */
    double shrink;           /* backtracking factor, default 0.5                         */
    int    max_backtracks;   /* default 30                                               */
    int    constrain_area;   /* total-area constraint row (Sec. 7.1.3), default 1        */
    int    constrain_volume; /* total-volume constraint row (Sec. 7.1.4), default 1      */
    double area_target;      /* NaN selects the area of the mesh at tp_problem_create    */
    double volume_target;    /* NaN selects the volume at tp_problem_create              */
    int    solver;           /* 0 (default): the direction with A~^{-1} in place of A_3^{-1};
                                1: A_3^{-1} by GMRES on A = B + B0 (Sec. 5.4;
                                tp_problem_sobolev_solve with the diagonal term)           */
    double solver_rtol;      /* GMRES relative residual, default 1e-4 (solver = 1); with
                                FP32 pair terms the attainable residual of smooth
                                right-hand sides (the constraint rows) lies near 1e-6     */
    int    solver_maxiter;   /* GMRES iterations at most, default 300 (solver = 1)        */
    double area_penalty;     /* w_A >= 0 of the potential w_A (A / A_0 - 1)^2 (Sec. 7.3.1),
                                A_0 = area_target; default 0                              */
    double volume_penalty;   /* w_V >= 0 of w_V (V / V_0 - 1)^2, V_0 = volume_target;
                                default 0.  With either weight > 0 the step minimises
                                the tangent-point energy plus the potentials: their
                                gradients join dE, the line search and E / E_new of the
                                report include them.  A weight > 0 with a target (or,
                                for a NaN target, an initial measure) of 0 gives
                                TP_E_INVALID_ARGUMENT: the potential divides by it       */
    int    barycenter_motion; /* 1: barycenter motions (Sec. 7.1.1): the solve removes every
                                component's mean, and the translation by minus the
                                vertex-area-weighted mean of dE (of the total objective)
                                over the component is added back to the direction; default 0 */
    int    warm_start;       /* 1 (default): the two Poisson solves of the preconditioner
                                start from the previous step's solutions of this problem
                                (same columns, one-launch preconditioned CG; the tolerance
                                stays relative to |b|); 0: from x = 0 (the paper's solve).
                                The first step of a problem always starts from zero       */
} tp_step_opts;

TP_API tp_status tp_step_opts_default(tp_step_opts* o);

typedef struct {
    double E;                /* energy at the start of the step                          */
    double E_new;            /* energy after the step (after the corrective projection)  */
    double grad_norm;        /* ||dE||_2                                                 */
    double slope;            /* dE . x (negative for a descent direction)                */
    double tau;              /* accepted step size                                       */
    int    backtracks;
    int    n_constraints;
    int    cg_iters[2];      /* the two Poisson solves' iterations; with solver = 1 the
                                GMRES iterations and the preconditioner's CG iterations  */
    double cg_relres[2];     /* their relative residuals; with solver = 1 GMRES's true
                                relative residual and 0                                  */
    double phi_before[2];    /* constraint values Phi(f) (area, volume; unused rows 0)   */
    double phi_trial[2];     /* Phi(f + tau x)                                           */
    double phi_after[2];     /* Phi after the corrective step                            */
    double t_ms[8];          /* device ms: [0] dE and right-hand sides, [1] first Poisson
                                solve, [2] preconditioner (both solves and the fractional
                                apply), [3] Schur system and direction, [4] line search,
                                [5] corrective projection and new energy, [6] whole step;
                                [7] number of problems whose launches this step shared    */
    int    warm_started;     /* 1 if the Poisson solves started from the previous step's
                                solutions                                                 */
} tp_step_report;

/* One projected, preconditioned descent step (the basic step of Sec. 3 with Sec. 5.3-5.4):
 * g = dE; J = active constraint rows; Y = A~^{-1} J^T, y_g = A~^{-1} g (one 3(1+k)-column
 * preconditioner application); S = J Y; x = -(y_g - Y S^{-1} J y_g); Armijo on E(f + tau x);
 * f <- f + tau x - Y S^{-1} Phi(f + tau x).  The problem's vertices are updated.
 * direction_out: optional device nV x 3 buffer receiving x (may be NULL).
 * report may be NULL. */
TP_API tp_status tp_precond_step(tp_problem* prob, const tp_step_opts* opts, tp_step_report* report,
                          double* direction_out);

/* Descent steps of n problems in one call (continuous batching of steps, not in the
 * paper): every phase of the step above runs for all problems before the next, the
 * all-pairs work of a phase in shared launches and the Poisson solves in shared
 * cooperative launches.  Each problem's arithmetic is that of tp_precond_step on it alone,
 * so its vertices and report are bit-identical to a step taken alone.  The problems must
 * be distinct and created on the same device and stream; problems that differ in
 * precision, exponents, sigma or number of active constraints run as separate groups.
 * opts: n entries or NULL (defaults); reports, statuses: n entries or NULL.  Returns TP_OK
 * when every problem succeeded, else the first problem's failure (statuses has all). */
TP_API tp_status tp_batch_step(tp_problem* const* probs, int n, const tp_step_opts* opts,
                               tp_step_report* reports, tp_status* statuses);

/* Device memory (bytes) the problem currently holds (its resident state and work arrays;
 * grows on first use of each call). */
TP_API tp_status tp_problem_device_bytes(const tp_problem* prob, uint64_t* bytes);

/* Upper bound of the device memory a problem with nV vertices, nF faces, largest vertex
 * degree max_degree and ncomp connected components holds after descent steps with
 * n_constraints (0..2) active constraint rows, for admission against a memory budget.
 * Uses the current device's pair-kernel plans.  Covers the default step (solver 0); the
 * GMRES solve (2 (restart + 1) nV k doubles of Krylov vectors and its work arrays), an
 * obstacle (32 B per obstacle face, 64 B per surface face) and barycenter motions (8 B
 * per vertex) come on top. */
TP_API tp_status tp_estimate_device_bytes(int64_t nV, int64_t nF, int max_degree, int ncomp,
                                          const tp_params* params, int n_constraints,
                                          uint64_t* bytes);

/* Barnes-Hut (params.theta > 0): E and dE of every energy / gradient / step call of the
 * problem use E_BH (Sec. 4.1): faces sorted by the Morton code of their barycenters (10
 * bits per coordinate on the barycenters' bounding box, ties by face index), leaves of
 * leaf_size consecutive faces, a perfect binary tree over the leaves; node I is
 * admissible for face S when max(r_S^2, r_I^2) < theta^2 dist^2 (r_S: largest distance
 * from X_S to a corner of S, r_I: from X_I = area-weighted barycenter to a corner of I's
 * box, dist: distance between the vertex boxes of S and I); admissible nodes contribute
 * K(X_S, N_S; X_I) a_S a_I, opened leaves their exact terms.  dE is the exact differential
 * of E_BH with the interaction lists held fixed (Sec. 4.2).  The fractional apply (every
 * L^sigma product: tp_fractional_apply, the preconditioner, the step) uses the same tree
 * and lists on the kernel matrix of Sec. 5.1.1: an admissible node I adds
 * |X_S - X_I|^-(2 sigma + 2) (a_I ubar_S - sum_{T in I} a_T ubar_T), an opened leaf its exact
 * terms (face sums only, deterministic).  The Poisson solves are unchanged.  This call
 * reports the numbers of far (node) and near (face) terms of the problem's last
 * Barnes-Hut energy evaluation. */
TP_API tp_status tp_problem_bh_stats(tp_problem* prob, int64_t* far_terms, int64_t* near_terms);

/* Numbers of admissible (rank-one) and inadmissible (exact leaf) blocks of the problem's
 * last block cluster tree (params.chi > 0; zeros before the first hierarchical product). */
TP_API tp_status tp_problem_bct_stats(tp_problem* prob, int64_t* admissible, int64_t* inadmissible);

/* ----------------------------------------------------------------- remeshing */

/* Dynamic remeshing (Sec. 6) of a triangle mesh between descent steps, on the host: one
 * pass of edge splits (edges longer than 1.5 L0 at their midpoint), one pass of edge
 * collapses (edges shorter than 0.5 L0 to their midpoint, refused where the link
 * condition fails or a remaining face around either end would turn its normal over),
 * then `iterations` rounds of Delaunay edge flips (interior edges whose opposite angles
 * sum to more than pi; repeated sweeps, at most 64) each followed by one step of
 * tangential smoothing: a vertex moves by rho times the area-weighted mean of (face
 * circumcenter - vertex) over its faces, projected onto the plane orthogonal to its
 * area-weighted normal; vertices on boundary edges stay.  Every choice follows the
 * sorted order of the edges (as vertex pairs), so the result depends on the mesh alone.
 * V: nV x 3 FP64 row-major, F: nF x 3 int32 (host memory, read only).  The result is
 * written to V_out (cap_V x 3) and F_out (cap_F x 3), caller-owned host buffers, and its
 * sizes to *nV_out, *nF_out; surviving vertices and faces keep their relative order and
 * faces their orientation.  If a capacity is too small (or V_out / F_out is NULL) the
 * sizes are still reported and TP_E_INVALID_ARGUMENT is returned: call again with room
 * (nV + the number of edges longer than 1.5 L0, at most, before smoothing and flips).
 * Errors: TP_E_INVALID_ARGUMENT (NULL inputs, nV < 3, nF < 1, L0 <= 0, iterations < 0,
 * rho outside [0, 1)), TP_E_BAD_INDEX (face index outside [0, nV)), TP_E_NONFINITE
 * (non-finite coordinates).  No device work; thread-safe.  The mesh's problem (its
 * incidence, sparsity and trees) is rebuilt by creating a new tp_problem from the result. */
TP_API tp_status tp_remesh(const double* V, int64_t nV, const int32_t* F, int64_t nF, double L0, int iterations,
                           double rho, double* V_out, int64_t cap_V, int32_t* F_out, int64_t cap_F,
                           int64_t* nV_out, int64_t* nF_out);

/* ------------------------------------------------------------------- diagnostics */

/* Message describing the last error of the calling thread ("" if none). */
TP_API const char* tp_last_error(void);

/* Device memory of the library.  By default every device buffer (resident problem state,
 * work arrays, temporaries of the stateless calls) comes from hipMalloc.  With an
 * allocator registered, every device buffer allocated afterwards comes from
 * alloc(bytes, stream, user) -- stream is the hipStream_t the buffer is first used on --
 * and is returned with free_(ptr, bytes, stream, user); a NULL result of alloc is
 * TP_E_OUT_OF_MEMORY.  This lets the caller's allocator (for example PyTorch's caching
 * allocator) own all device memory.  Pinned host buffers for read-backs still use
 * hipHostMalloc.  alloc = free_ = NULL restores hipMalloc.  The registration is
 * process-global and may change only while no buffer of the registered allocator is
 * alive (TP_E_INVALID_ARGUMENT otherwise): register before creating problems, and destroy
 * them before unregistering.  Both functions must be callable from any thread that calls
 * the library and must not call back into it. */
typedef void* (*tp_alloc_fn)(size_t bytes, void* stream, void* user);
typedef void (*tp_free_fn)(void* ptr, size_t bytes, void* stream, void* user);
TP_API tp_status tp_set_allocator(tp_alloc_fn alloc, tp_free_fn free_, void* user);

/* Kernel timing for roofline reports.  When enabled, every all-pairs kernel launch is
 * bracketed by HIP events recorded on the stream it runs on; the elapsed device time,
 * the number of ordered face pairs it covered and the launch count are accumulated per
 * kind: 0 = energy, 1 = energy + differential, 2 = fractional apply, 3 = the inner-product
 * operator A (tp_sobolev_apply; the pair kernel alone).  Process-global.  Timing never
 * makes the host wait: the events are read when tp_profile_get or tp_profile_reset is
 * called, which wait for the launches still running. */
typedef struct {
    double  ms_total;      /* summed device time of the launches                        */
    double  pairs_total;   /* summed ordered pairs S != T evaluated (columns not counted) */
    double  cols_total;    /* summed pairs x columns (fractional apply and operator A)   */
    int64_t launches;
} tp_kernel_stats;

TP_API tp_status tp_profile_enable(int on);
TP_API tp_status tp_profile_reset(void);
TP_API tp_status tp_profile_get(int kind, tp_kernel_stats* out);

#ifdef __cplusplus
}
#endif
#endif /* TPSURF_H */
