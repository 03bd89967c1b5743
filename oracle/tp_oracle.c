/*
 * tp_oracle.c -- plain FP64 CPU reference for the tangent-point hot path of
 * "Repulsive Surfaces" (Yu, Brakensiek, Schumacher, Crane 2021).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark may load this library.  It shares no code with the HIP path.
 *
 * Everything here is the paper's definition written out with plain loops in double
 * precision: no blocking, no fusion, no reordering of the sums beyond splitting the
 * outer sum over faces S into rows, which are reduced in increasing S order, so the
 * result does not depend on the number of OpenMP threads.
 *
 * Conventions: V is nV x 3 row-major double, F is nF x 3 int32 with 0-based vertex
 * indices.  A face S = (i, j, k) has edges e1 = f_j - f_i, e2 = f_k - f_i.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define EXPORT __attribute__((visibility("default")))

/* ------------------------------------------------------------------------- */
/* Face quantities (Sec. 3.1, eq. DiscreteTangentPointKernel and the text after
 * eq. DiscreteEnergy): barycenter X_S, area a_S, unit normal N_S.  The normal
 * enters only through the projector N N^T, so its sign is irrelevant (Sec. 2.1). */
static void face_quantities(const double* V, const int32_t* F, int64_t s,
                            double X[3], double N[3], double* a, double c[3])
{
    const double* fi = V + 3 * (int64_t)F[3 * s + 0];
    const double* fj = V + 3 * (int64_t)F[3 * s + 1];
    const double* fk = V + 3 * (int64_t)F[3 * s + 2];
    double e1[3], e2[3];
    for (int d = 0; d < 3; ++d) {
        X[d] = (fi[d] + fj[d] + fk[d]) / 3.0;
        e1[d] = fj[d] - fi[d];
        e2[d] = fk[d] - fi[d];
    }
    c[0] = e1[1] * e2[2] - e1[2] * e2[1];
    c[1] = e1[2] * e2[0] - e1[0] * e2[2];
    c[2] = e1[0] * e2[1] - e1[1] * e2[0];
    double cn = sqrt(c[0] * c[0] + c[1] * c[1] + c[2] * c[2]);
    *a = 0.5 * cn;
    for (int d = 0; d < 3; ++d) N[d] = c[d] / cn;
}

EXPORT void tpo_faces(const double* V, const int32_t* F, int64_t nF,
                      double* X, double* N, double* A)
{
    for (int64_t s = 0; s < nF; ++s) {
        double c[3];
        face_quantities(V, F, s, X + 3 * s, N + 3 * s, A + s, c);
    }
}

static void all_faces(const double* V, const int32_t* F, int64_t nF,
                      double* X, double* N, double* A, double* C)
{
    for (int64_t s = 0; s < nF; ++s)
        face_quantities(V, F, s, X + 3 * s, N + 3 * s, A + s, C + 3 * s);
}

/* ------------------------------------------------------------------------- */
/* Discrete tangent-point kernel (eq. DiscreteTangentPointKernel) with independent
 * exponents: K(S,T) = |P_S d|^alpha / |d|^beta, d = X_S - X_T, P_S = N_S N_S^T.
 * Since |N_S| = 1, |P_S d| = |N_S . d|.  The paper's choice is alpha = p, beta = 2p. */
static double tp_kernel(const double XS[3], const double NS[3], const double XT[3],
                        double alpha, double beta)
{
    double d[3] = {XS[0] - XT[0], XS[1] - XT[1], XS[2] - XT[2]};
    double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
    double q = NS[0] * d[0] + NS[1] * d[1] + NS[2] * d[2];
    return pow(fabs(q), alpha) * pow(r2, -0.5 * beta);
}

/* Partial derivatives of K(S,T) with respect to d = X_S - X_T and to N_S:
 *   dK/dd = alpha |q|^(alpha-1) sgn(q) |d|^-beta N_S - beta K |d|^-2 d,
 *   dK/dN = alpha |q|^(alpha-1) sgn(q) |d|^-beta d,       q = N_S . d.        */
static double tp_kernel_grad(const double XS[3], const double NS[3], const double XT[3],
                             double alpha, double beta, double dKdd[3], double dKdN[3])
{
    double d[3] = {XS[0] - XT[0], XS[1] - XT[1], XS[2] - XT[2]};
    double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
    double q = NS[0] * d[0] + NS[1] * d[1] + NS[2] * d[2];
    double rb = pow(r2, -0.5 * beta);
    double K = pow(fabs(q), alpha) * rb;
    double sq = (q > 0.0) ? 1.0 : ((q < 0.0) ? -1.0 : 0.0);
    double c1 = alpha * pow(fabs(q), alpha - 1.0) * sq * rb;
    double c2 = beta * K / r2;
    for (int m = 0; m < 3; ++m) {
        dKdd[m] = c1 * NS[m] - c2 * d[m];
        dKdN[m] = c1 * d[m];
    }
    return K;
}

/* ------------------------------------------------------------------------- */
/* Energy (eq. DiscreteEnergy): E = sum_S sum_{T != S} K(S,T) a_S a_T.
 * The diagonal S = T is excluded: K(S,S) is 0/0, and the kernel matrix of
 * Sec. 5.1 carries the factor (1 - delta_ST).
 * E depends on the mesh only through the face quantities (X, N, a), so the sum is
 * written on those: Erow[s - s0] = sum_{T != S} K(S,T) a_S a_T for S in [s0, s1),
 * X and N are nF x 3 row-major.                                                   */
EXPORT void tpo_energy_faces_rows(const double* X, const double* N, const double* A, int64_t nF,
                                  double alpha, double beta, int64_t s0, int64_t s1, double* Erow)
{
#pragma omp parallel for schedule(dynamic, 8)
    for (int64_t S = s0; S < s1; ++S) {
        double row = 0.0;
        for (int64_t T = 0; T < nF; ++T) {
            if (T == S) continue;
            row += tp_kernel(X + 3 * S, N + 3 * S, X + 3 * T, alpha, beta) * A[S] * A[T];
        }
        Erow[S - s0] = row;
    }
}

EXPORT double tpo_energy_faces(const double* X, const double* N, const double* A, int64_t nF,
                               double alpha, double beta)
{
    double* Erow = malloc(sizeof(double) * nF);
    tpo_energy_faces_rows(X, N, A, nF, alpha, beta, 0, nF, Erow);
    double E = 0.0;
    for (int64_t S = 0; S < nF; ++S) E += Erow[S];
    free(Erow);
    return E;
}

EXPORT double tpo_energy(const double* V, int64_t nV, const int32_t* F, int64_t nF,
                         double alpha, double beta)
{
    (void)nV;
    double* X = malloc(sizeof(double) * 3 * nF);
    double* N = malloc(sizeof(double) * 3 * nF);
    double* A = malloc(sizeof(double) * nF);
    double* C = malloc(sizeof(double) * 3 * nF);
    all_faces(V, F, nF, X, N, A, C);
    double E = tpo_energy_faces(X, N, A, nF, alpha, beta);
    free(X); free(N); free(A); free(C);
    return E;
}

/* ------------------------------------------------------------------------- */
/* Differential of E by the chain rule (text after eq. DiscreteEnergy).
 *
 * E depends on f only through the face quantities X, N, a.  For a face S, the terms
 * that involve S are the pairs (S,T) (S first: depends on X_S, N_S, a_S) and (T,S)
 * (S second: depends on X_S, a_S).  Summing their partial derivatives:
 *
 *   dE/dX_S = sum_T [ a_S a_T dK(S,T)/dd  -  a_T a_S dK(T,S)/dd' ]   (d' = X_T - X_S)
 *   dE/dN_S = sum_T   a_S a_T dK(S,T)/dN_S
 *   dE/da_S = sum_T [ K(S,T) a_T + K(T,S) a_T ]
 *
 * gface[7 s + 0..2] = dE/dX_S, [3..5] = dE/dN_S, [6] = dE/da_S for S in [s0, s1);
 * Erow[s - s0] as in tpo_energy_faces_rows.                                            */
static void gradient_row(const double* X, const double* N, const double* A, int64_t nF,
                         double alpha, double beta, int64_t S, double g[7], double* Erow)
{
    double gX[3] = {0, 0, 0}, gN[3] = {0, 0, 0}, ga = 0.0, row = 0.0;
    for (int64_t T = 0; T < nF; ++T) {
        if (T == S) continue;
        double dKdd[3], dKdN[3], dKdd_r[3], dKdN_r[3];
        double K = tp_kernel_grad(X + 3 * S, N + 3 * S, X + 3 * T, alpha, beta, dKdd, dKdN);
        double Kr = tp_kernel_grad(X + 3 * T, N + 3 * T, X + 3 * S, alpha, beta, dKdd_r, dKdN_r);
        double w = A[S] * A[T];
        for (int m = 0; m < 3; ++m) {
            gX[m] += w * dKdd[m] - w * dKdd_r[m];
            gN[m] += w * dKdN[m];
        }
        ga += K * A[T] + Kr * A[T];
        row += K * w;
    }
    for (int m = 0; m < 3; ++m) { g[m] = gX[m]; g[3 + m] = gN[m]; }
    g[6] = ga;
    if (Erow) *Erow = row;
}

EXPORT void tpo_gradient_rows(const double* V, int64_t nV, const int32_t* F, int64_t nF,
                              double alpha, double beta, int64_t s0, int64_t s1,
                              double* gface, double* Erow)
{
    (void)nV;
    double* X = malloc(sizeof(double) * 3 * nF);
    double* N = malloc(sizeof(double) * 3 * nF);
    double* A = malloc(sizeof(double) * nF);
    double* C = malloc(sizeof(double) * 3 * nF);
    all_faces(V, F, nF, X, N, A, C);
#pragma omp parallel for schedule(dynamic, 8)
    for (int64_t S = s0; S < s1; ++S)
        gradient_row(X, N, A, nF, alpha, beta, S, gface + 7 * (S - s0), Erow ? Erow + (S - s0) : NULL);
    free(X); free(N); free(A); free(C);
}

/* Same per-face sums for an explicit list of faces rows[0..nrows). */
EXPORT void tpo_gradient_rowlist(const double* V, int64_t nV, const int32_t* F, int64_t nF,
                                 double alpha, double beta, const int64_t* rows, int64_t nrows,
                                 double* gface, double* Erow)
{
    (void)nV;
    double* X = malloc(sizeof(double) * 3 * nF);
    double* N = malloc(sizeof(double) * 3 * nF);
    double* A = malloc(sizeof(double) * nF);
    double* C = malloc(sizeof(double) * 3 * nF);
    all_faces(V, F, nF, X, N, A, C);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t q = 0; q < nrows; ++q)
        gradient_row(X, N, A, nF, alpha, beta, rows[q], gface + 7 * q, Erow ? Erow + q : NULL);
    free(X); free(N); free(A); free(C);
}

/* Chain rule from face quantities to vertex positions.
 *   X_S = (f_i + f_j + f_k)/3                      -> each corner gets dE/dX_S / 3
 *   c = e1 x e2, a_S = |c|/2, N_S = c/|c|          -> g_c = (I - N N^T) dE/dN_S / |c| + dE/da_S N_S / 2
 *   dc = (df_j - df_i) x e2 + e1 x (df_k - df_i)   -> df_j: e2 x g_c,  df_k: g_c x e1,  df_i: -(both)
 * Faces are visited in increasing order, so the vertex sums are deterministic. */
EXPORT void tpo_face_to_vertex(const double* V, int64_t nV, const int32_t* F, int64_t nF,
                               const double* gface, double* dE)
{
    memset(dE, 0, sizeof(double) * 3 * nV);
    for (int64_t S = 0; S < nF; ++S) {
        double X[3], N[3], a, c[3];
        face_quantities(V, F, S, X, N, &a, c);
        const double* g = gface + 7 * S;
        const double* fi = V + 3 * (int64_t)F[3 * S + 0];
        const double* fj = V + 3 * (int64_t)F[3 * S + 1];
        const double* fk = V + 3 * (int64_t)F[3 * S + 2];
        double e1[3], e2[3];
        for (int m = 0; m < 3; ++m) { e1[m] = fj[m] - fi[m]; e2[m] = fk[m] - fi[m]; }
        double cn = 2.0 * a;
        double ndg = N[0] * g[3] + N[1] * g[4] + N[2] * g[5];
        double gc[3];
        for (int m = 0; m < 3; ++m) gc[m] = (g[3 + m] - N[m] * ndg) / cn + 0.5 * g[6] * N[m];
        double dj[3] = {e2[1] * gc[2] - e2[2] * gc[1], e2[2] * gc[0] - e2[0] * gc[2], e2[0] * gc[1] - e2[1] * gc[0]};
        double dk[3] = {gc[1] * e1[2] - gc[2] * e1[1], gc[2] * e1[0] - gc[0] * e1[2], gc[0] * e1[1] - gc[1] * e1[0]};
        int64_t vi = F[3 * S + 0], vj = F[3 * S + 1], vk = F[3 * S + 2];
        for (int m = 0; m < 3; ++m) {
            double gx = g[m] / 3.0;
            dE[3 * vi + m] += gx - dj[m] - dk[m];
            dE[3 * vj + m] += gx + dj[m];
            dE[3 * vk + m] += gx + dk[m];
        }
    }
}

EXPORT double tpo_gradient(const double* V, int64_t nV, const int32_t* F, int64_t nF,
                           double alpha, double beta, double* dE)
{
    double* gface = malloc(sizeof(double) * 7 * nF);
    double* Erow = malloc(sizeof(double) * nF);
    tpo_gradient_rows(V, nV, F, nF, alpha, beta, 0, nF, gface, Erow);
    tpo_face_to_vertex(V, nV, F, nF, gface, dE);
    double E = 0.0;
    for (int64_t S = 0; S < nF; ++S) E += Erow[S];
    free(gface); free(Erow);
    return E;
}

/* ------------------------------------------------------------------------- */
/* Fractional operator applied to k columns (eq. DiscreteLaplacianQuartic):
 *
 *   (L u)_i = sum_{S != T} (phi_i(S) - phi_i(T)) (ubar(S) - ubar(T)) |X_S - X_T|^-(2 sigma + 2) a_S a_T
 *
 * where ubar(S) = sum_j phi_j(S) u_j is the average of u over the corners of S
 * (phi_j(S) = 1/3 for the corners of S, 0 otherwise).  The part carrying phi_i(T)
 * equals the part carrying phi_i(S) after renaming S <-> T (the rest of the summand is
 * antisymmetric times symmetric), so
 *
 *   (L u)_i = 2 sum_S phi_i(S) w(S),   w(S) = sum_{T != S} (ubar(S) - ubar(T)) |X_S - X_T|^-(2 sigma + 2) a_S a_T.
 *
 * u and Lu are nV x k row-major.  wrow[(s - s0) k + c] = w(S) for S in [s0, s1). */
static void fractional_prepare(const double* V, const int32_t* F, int64_t nF, const double* u, int k,
                               double** X, double** A, double** ub)
{
    double* N = malloc(sizeof(double) * 3 * nF);
    double* C = malloc(sizeof(double) * 3 * nF);
    *X = malloc(sizeof(double) * 3 * nF);
    *A = malloc(sizeof(double) * nF);
    *ub = malloc(sizeof(double) * nF * k);
    all_faces(V, F, nF, *X, N, *A, C);
    for (int64_t S = 0; S < nF; ++S)
        for (int c = 0; c < k; ++c)
            (*ub)[S * k + c] = (u[(int64_t)F[3 * S] * k + c] + u[(int64_t)F[3 * S + 1] * k + c] +
                                u[(int64_t)F[3 * S + 2] * k + c]) / 3.0;
    free(N); free(C);
}

static void fractional_row(const double* X, const double* A, const double* ub, int64_t nF, int k,
                           double sigma, int64_t S, double* out)
{
    double acc[64];
    double expo = -(2.0 * sigma + 2.0) * 0.5;  /* |d|^-(2 sigma + 2) = (|d|^2)^expo */
    for (int c = 0; c < k; ++c) acc[c] = 0.0;
    for (int64_t T = 0; T < nF; ++T) {
        if (T == S) continue;
        double d0 = X[3 * S] - X[3 * T], d1 = X[3 * S + 1] - X[3 * T + 1], d2 = X[3 * S + 2] - X[3 * T + 2];
        double h = pow(d0 * d0 + d1 * d1 + d2 * d2, expo) * A[S] * A[T];
        for (int c = 0; c < k; ++c) acc[c] += (ub[S * k + c] - ub[T * k + c]) * h;
    }
    for (int c = 0; c < k; ++c) out[c] = acc[c];
}

EXPORT void tpo_fractional_rows(const double* V, int64_t nV, const int32_t* F, int64_t nF,
                                double sigma, const double* u, int k,
                                int64_t s0, int64_t s1, double* wrow)
{
    (void)nV;
    double *X, *A, *ub;
    fractional_prepare(V, F, nF, u, k, &X, &A, &ub);
#pragma omp parallel for schedule(dynamic, 8)
    for (int64_t S = s0; S < s1; ++S) fractional_row(X, A, ub, nF, k, sigma, S, wrow + (S - s0) * k);
    free(X); free(A); free(ub);
}

EXPORT void tpo_fractional_rowlist(const double* V, int64_t nV, const int32_t* F, int64_t nF,
                                   double sigma, const double* u, int k, const int64_t* rows,
                                   int64_t nrows, double* wrow)
{
    (void)nV;
    double *X, *A, *ub;
    fractional_prepare(V, F, nF, u, k, &X, &A, &ub);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t q = 0; q < nrows; ++q) fractional_row(X, A, ub, nF, k, sigma, rows[q], wrow + q * k);
    free(X); free(A); free(ub);
}

/* (L u)_i = 2 sum_S phi_i(S) w(S) with phi_i(S) = 1/3 on the corners of S. */
EXPORT void tpo_fractional_gather(const int32_t* F, int64_t nF, int64_t nV, const double* w, int k,
                                  double* Lu)
{
    memset(Lu, 0, sizeof(double) * nV * k);
    for (int64_t S = 0; S < nF; ++S)
        for (int corner = 0; corner < 3; ++corner) {
            int64_t i = F[3 * S + corner];
            for (int c = 0; c < k; ++c) Lu[i * k + c] += 2.0 * (w[S * k + c] / 3.0);
        }
}

EXPORT int tpo_fractional_apply(const double* V, int64_t nV, const int32_t* F, int64_t nF,
                                double sigma, const double* u, int k, double* Lu)
{
    if (k < 1 || k > 64) return 1;
    double* w = malloc(sizeof(double) * nF * k);
    tpo_fractional_rows(V, nV, F, nF, sigma, u, k, 0, nF, w);
    tpo_fractional_gather(F, nF, nV, w, k, Lu);
    free(w);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* The operator A = B + B0 of the inner product (Sec. 2.4, the high- and low-order terms;
 * discretized in Sec. 3.2.1, eqs. DiscreteHighOrderTerm and DiscreteLowOrderTerm) applied to
 * k columns, with sigma = s - 1 so that |d|^-(2 sigma + 2) = |d|^-2s:
 *
 *   (B u)_i  = sum_{S != T} < D phi_i(S) - D phi_i(T), D u(S) - D u(T) > |d|^-2s a_S a_T
 *   (B0 u)_i = sum_{S != T} (phibar_i(S) - phibar_i(T)) (ubar(S) - ubar(T)) |d|^-2s K2(S,T) a_S a_T
 *
 * d = X_S - X_T; K2(S,T) = (N_S . d)^2 / |d|^4 is the discrete tangent-point kernel with
 * exponents 2 and 4; D u(S) is the gradient of the piecewise linear u on S,
 * D phi_i(S) = N_S x (f_k - f_j) / (2 a_S) for the corners (i, j, k) of S taken cyclically,
 * i.e. c_S x (f_k - f_j) / |c_S|^2 with c_S = (f_j - f_i) x (f_k - f_i).  Renaming S <-> T in
 * the parts that carry phi_i(T) (as for the fractional operator):
 *
 *   (B u)_i  = 2 sum_S < D phi_i(S), zB(S) >,  zB(S) = sum_{T != S} |d|^-2s a_S a_T (D u(S) - D u(T))
 *   (B0 u)_i = 2 sum_S phibar_i(S) z0(S),
 *              z0(S) = sum_{T != S} |d|^-2s (K2(S,T) + K2(T,S)) / 2 a_S a_T (ubar(S) - ubar(T)),
 *
 * where only the symmetric part of K2 survives because the rest of the summand is
 * symmetric in (S, T).  zrow[(S - s0) 4k + 4c + m] = zB(S)[c][m] for m < 3, z0(S)[c] for m = 3. */
static void face_gradients(const double* V, const int32_t* F, int64_t nF, const double* u, int k,
                           double* Du /* nF x k x 3 */)
{
    for (int64_t S = 0; S < nF; ++S) {
        double X[3], N[3], a, c[3];
        face_quantities(V, F, S, X, N, &a, c);
        double c2 = c[0] * c[0] + c[1] * c[1] + c[2] * c[2];
        for (int cc = 0; cc < k; ++cc)
            for (int m = 0; m < 3; ++m) Du[(S * k + cc) * 3 + m] = 0.0;
        for (int corner = 0; corner < 3; ++corner) {
            const double* fj = V + 3 * (int64_t)F[3 * S + (corner + 1) % 3];
            const double* fk = V + 3 * (int64_t)F[3 * S + (corner + 2) % 3];
            double e[3] = {fk[0] - fj[0], fk[1] - fj[1], fk[2] - fj[2]};
            double g[3] = {(c[1] * e[2] - c[2] * e[1]) / c2, (c[2] * e[0] - c[0] * e[2]) / c2,
                           (c[0] * e[1] - c[1] * e[0]) / c2};
            int64_t i = F[3 * S + corner];
            for (int cc = 0; cc < k; ++cc)
                for (int m = 0; m < 3; ++m) Du[(S * k + cc) * 3 + m] += u[i * k + cc] * g[m];
        }
    }
}

EXPORT void tpo_face_gradients(const double* V, const int32_t* F, int64_t nF, const double* u, int k,
                               double* Du)
{
    face_gradients(V, F, nF, u, k, Du);
}

static void sobolev_row(const double* X, const double* N, const double* A, const double* ub,
                        const double* Du, int64_t nF, int k, double s, int64_t S, double* out)
{
    double accB[64 * 3], acc0[64];
    for (int c = 0; c < 3 * k; ++c) accB[c] = 0.0;
    for (int c = 0; c < k; ++c) acc0[c] = 0.0;
    for (int64_t T = 0; T < nF; ++T) {
        if (T == S) continue;
        double d[3] = {X[3 * S] - X[3 * T], X[3 * S + 1] - X[3 * T + 1], X[3 * S + 2] - X[3 * T + 2]};
        double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
        double h = pow(r2, -s) * A[S] * A[T];   /* |d|^-2s a_S a_T */
        double qS = N[3 * S] * d[0] + N[3 * S + 1] * d[1] + N[3 * S + 2] * d[2];
        double qT = N[3 * T] * d[0] + N[3 * T + 1] * d[1] + N[3 * T + 2] * d[2];
        double k2 = 0.5 * (qS * qS / (r2 * r2) + qT * qT / (r2 * r2));
        for (int c = 0; c < k; ++c) {
            for (int m = 0; m < 3; ++m)
                accB[3 * c + m] += (Du[(S * k + c) * 3 + m] - Du[(T * k + c) * 3 + m]) * h;
            acc0[c] += (ub[S * k + c] - ub[T * k + c]) * h * k2;
        }
    }
    for (int c = 0; c < k; ++c) {
        for (int m = 0; m < 3; ++m) out[4 * c + m] = accB[3 * c + m];
        out[4 * c + 3] = acc0[c];
    }
}

static void sobolev_prepare(const double* V, const int32_t* F, int64_t nF, const double* u, int k,
                            double** X, double** N, double** A, double** ub, double** Du)
{
    double* C = malloc(sizeof(double) * 3 * nF);
    *X = malloc(sizeof(double) * 3 * nF);
    *N = malloc(sizeof(double) * 3 * nF);
    *A = malloc(sizeof(double) * nF);
    *ub = malloc(sizeof(double) * nF * k);
    *Du = malloc(sizeof(double) * nF * k * 3);
    all_faces(V, F, nF, *X, *N, *A, C);
    for (int64_t S = 0; S < nF; ++S)
        for (int c = 0; c < k; ++c)
            (*ub)[S * k + c] = (u[(int64_t)F[3 * S] * k + c] + u[(int64_t)F[3 * S + 1] * k + c] +
                                u[(int64_t)F[3 * S + 2] * k + c]) / 3.0;
    face_gradients(V, F, nF, u, k, *Du);
    free(C);
}

EXPORT void tpo_sobolev_rowlist(const double* V, int64_t nV, const int32_t* F, int64_t nF, double s,
                                const double* u, int k, const int64_t* rows, int64_t nrows, double* zrow)
{
    (void)nV;
    double *X, *N, *A, *ub, *Du;
    sobolev_prepare(V, F, nF, u, k, &X, &N, &A, &ub, &Du);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t q = 0; q < nrows; ++q) sobolev_row(X, N, A, ub, Du, nF, k, s, rows[q], zrow + q * 4 * k);
    free(X); free(N); free(A); free(ub); free(Du);
}

/* (A u)_i = 2 sum_S (< D phi_i(S), zB(S) > + phibar_i(S) z0(S)) over the faces S with corner i. */
EXPORT void tpo_sobolev_gather(const double* V, const int32_t* F, int64_t nF, int64_t nV, const double* z,
                               int k, double* Au)
{
    memset(Au, 0, sizeof(double) * nV * k);
    for (int64_t S = 0; S < nF; ++S) {
        double X[3], N[3], a, c[3];
        face_quantities(V, F, S, X, N, &a, c);
        double c2 = c[0] * c[0] + c[1] * c[1] + c[2] * c[2];
        for (int corner = 0; corner < 3; ++corner) {
            const double* fj = V + 3 * (int64_t)F[3 * S + (corner + 1) % 3];
            const double* fk = V + 3 * (int64_t)F[3 * S + (corner + 2) % 3];
            double e[3] = {fk[0] - fj[0], fk[1] - fj[1], fk[2] - fj[2]};
            double g[3] = {(c[1] * e[2] - c[2] * e[1]) / c2, (c[2] * e[0] - c[0] * e[2]) / c2,
                           (c[0] * e[1] - c[1] * e[0]) / c2};
            int64_t i = F[3 * S + corner];
            for (int cc = 0; cc < k; ++cc) {
                const double* zc = z + S * 4 * k + 4 * cc;
                Au[i * k + cc] += 2.0 * (g[0] * zc[0] + g[1] * zc[1] + g[2] * zc[2] + zc[3] / 3.0);
            }
        }
    }
}

EXPORT int tpo_sobolev_apply(const double* V, int64_t nV, const int32_t* F, int64_t nF, double s,
                             const double* u, int k, double* Au)
{
    if (k < 1 || k > 64) return 1;
    double* z = malloc(sizeof(double) * nF * 4 * k);
    int64_t* rows = malloc(sizeof(int64_t) * nF);
    for (int64_t S = 0; S < nF; ++S) rows[S] = S;
    tpo_sobolev_rowlist(V, nV, F, nF, s, u, k, rows, nF, z);
    tpo_sobolev_gather(V, F, nF, nV, z, k, Au);
    free(z); free(rows);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Static obstacle potential (Sec. 7.3.2): the obstacle's potential sum_S a_O(S) |X_O(S) - x|^-p
 * evaluated at the barycenter of every surface face T and integrated over T:
 *   E_obs = sum_T a_T phi(T),  phi(T) = sum_S a_O(S) |X_O(S) - X_T|^-p.
 * Its differential with respect to the surface vertices, by the chain rule through X_T
 * (d X_T / d f_i = I/3 for the corners) and a_T (d a_T / d f_i = N_T x (f_k - f_j) / 2 for
 * the corners i, j, k of T in cyclic order).  dE (nV x 3) may be NULL. */
EXPORT double tpo_obstacle(const double* V, int64_t nV, const int32_t* F, int64_t nF, const double* Vo,
                           const int32_t* Fo, int64_t nFo, double p, double* dE)
{
    double* XO = malloc(sizeof(double) * 3 * nFo);
    double* AO = malloc(sizeof(double) * nFo);
    for (int64_t S = 0; S < nFo; ++S) {
        double N[3], c[3];
        face_quantities(Vo, Fo, S, XO + 3 * S, N, AO + S, c);
    }
    if (dE) memset(dE, 0, sizeof(double) * 3 * nV);
    double E = 0.0;
    for (int64_t T = 0; T < nF; ++T) {
        double X[3], N[3], a, c[3];
        face_quantities(V, F, T, X, N, &a, c);
        double phi = 0.0, g[3] = {0.0, 0.0, 0.0};
        for (int64_t S = 0; S < nFo; ++S) {
            double d[3] = {X[0] - XO[3 * S], X[1] - XO[3 * S + 1], X[2] - XO[3 * S + 2]};
            double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
            double w = AO[S] * pow(r2, -0.5 * p);
            phi += w;
            for (int m = 0; m < 3; ++m) g[m] += -p * w / r2 * d[m];
        }
        E += a * phi;
        if (!dE) continue;
        for (int corner = 0; corner < 3; ++corner) {
            const double* fj = V + 3 * (int64_t)F[3 * T + (corner + 1) % 3];
            const double* fk = V + 3 * (int64_t)F[3 * T + (corner + 2) % 3];
            double e[3] = {fk[0] - fj[0], fk[1] - fj[1], fk[2] - fj[2]};
            double da[3] = {0.5 * (N[1] * e[2] - N[2] * e[1]), 0.5 * (N[2] * e[0] - N[0] * e[2]),
                            0.5 * (N[0] * e[1] - N[1] * e[0])};
            int64_t i = F[3 * T + corner];
            for (int m = 0; m < 3; ++m) dE[3 * i + m] += a * g[m] / 3.0 + phi * da[m];
        }
    }
    free(XO); free(AO);
    return E;
}

/* ------------------------------------------------------------------------- */
/* Barnes-Hut approximation of the energy (Sec. 4.1) and its differential (Sec. 4.2).
 *
 * Tree (reading: the paper names a BVH with at most 8 faces per leaf and leaves the
 * build open).  Faces are sorted by the 30-bit Morton code of their barycenter, each
 * coordinate quantized to 10 bits on the bounding box of all barycenters
 * (q = min(1023, floor(1024 (x - lo) / (hi - lo)))), ties broken by face index.  Leaves
 * hold `leaf` consecutive sorted faces; the internal nodes form a perfect binary tree over
 * the leaves in heap order (node 1 is the root, node i has children 2i and 2i + 1, the
 * leaves are nodes P .. 2P - 1 for P the smallest power of two >= the number of leaves;
 * the leaves past the last face are empty).  A node I carries a_I = sum of its faces'
 * areas, X_I = (sum a_T X_T) / a_I (sums in sorted order, children left then right) and
 * the bounding box of its faces' vertices.
 *
 * Admissibility (reading: the printed inequality lacks theta): node I is admissible for
 * face S when max(r_S^2, r_I^2) < theta^2 dist^2, with r_S the largest distance from X_S
 * to a corner of S, r_I the largest distance from X_I to a corner of the box of I and
 * dist the distance between the box of S's vertices and the box of I.  theta = 0 admits
 * nothing and gives the exact sum.
 *
 * Traversal from the root, depth first, left child first: an admissible node adds
 * K(X_S, N_S; X_I) a_S a_I; a leaf that is not admissible adds the exact terms
 * K(S,T) a_S a_T of its faces T != S; other nodes are opened.  E_BH is the sum over S.
 *
 * Differential (reading: the exact gradient of E_BH with every face's list of admissible
 * nodes and opened leaves held fixed).  Each term w K(X_S, N_S; Y) a_S with target Y,
 * w = a_T or a_I, gives S: dX += a_S w dK/dd, dN += a_S w dK/dN, da += w K, and the target:
 * dY -= a_S w dK/dd, dw += a_S K.  A node's (dX_I, da_I) reach its member faces through
 * X_I = sum a_T X_T / a_I and a_I = sum a_T:
 *   dX_T += (a_T / a_I) dX_I,   da_T += da_I + (X_T - X_I) . dX_I / a_I.
 * All arithmetic is FP64; sums run in face order, then node order (deterministic).       */

typedef struct {
    int64_t nF, nleaf, P;
    int leaf;
    int64_t* order;        /* sorted position -> face */
    double* lo;            /* [2P][3] node boxes */
    double* hi;
    double* a;             /* [2P] */
    double* X;             /* [2P][3] */
    double* r2;            /* [2P] */
    double* flo;           /* [nF][3] face boxes */
    double* fhi;
    double* fr2;           /* [nF] r_S^2 */
} bh_tree;

static uint32_t bh_spread10(uint32_t v)
{
    uint32_t out = 0;
    for (int b = 0; b < 10; ++b) out |= ((v >> b) & 1u) << (3 * b);
    return out;
}

static uint32_t bh_quant(double x, double lo, double hi)
{
    if (!(hi > lo)) return 0;
    double t = floor(1024.0 * ((x - lo) / (hi - lo)));
    if (t < 0.0) t = 0.0;
    if (t > 1023.0) t = 1023.0;
    return (uint32_t)t;
}

static const uint64_t* bh_sort_keys;
static int bh_cmp(const void* pa, const void* pb)
{
    uint64_t ka = bh_sort_keys[*(const int64_t*)pa], kb = bh_sort_keys[*(const int64_t*)pb];
    return ka < kb ? -1 : (ka > kb ? 1 : 0);
}

static void bh_build(const double* V, const int32_t* F, int64_t nF, const double* X, const double* A,
                     int leaf, bh_tree* T)
{
    T->nF = nF;
    T->leaf = leaf;
    T->nleaf = (nF + leaf - 1) / leaf;
    T->P = 1;
    while (T->P < T->nleaf) T->P *= 2;
    const int64_t M = 2 * T->P;
    T->order = malloc(sizeof(int64_t) * nF);
    T->lo = malloc(sizeof(double) * 3 * M);
    T->hi = malloc(sizeof(double) * 3 * M);
    T->a = calloc(M, sizeof(double));
    T->X = calloc(3 * M, sizeof(double));
    T->r2 = calloc(M, sizeof(double));
    T->flo = malloc(sizeof(double) * 3 * nF);
    T->fhi = malloc(sizeof(double) * 3 * nF);
    T->fr2 = malloc(sizeof(double) * nF);
    /* face boxes and r_S^2 */
    for (int64_t s = 0; s < nF; ++s) {
        double best = 0.0;
        for (int m = 0; m < 3; ++m) { T->flo[3 * s + m] = INFINITY; T->fhi[3 * s + m] = -INFINITY; }
        for (int c = 0; c < 3; ++c) {
            const double* v = V + 3 * (int64_t)F[3 * s + c];
            double d2 = 0.0;
            for (int m = 0; m < 3; ++m) {
                if (v[m] < T->flo[3 * s + m]) T->flo[3 * s + m] = v[m];
                if (v[m] > T->fhi[3 * s + m]) T->fhi[3 * s + m] = v[m];
                double dm = v[m] - X[3 * s + m];
                d2 += dm * dm;
            }
            if (d2 > best) best = d2;
        }
        T->fr2[s] = best;
    }
    /* Morton order */
    double blo[3] = {INFINITY, INFINITY, INFINITY}, bhi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int64_t s = 0; s < nF; ++s)
        for (int m = 0; m < 3; ++m) {
            if (X[3 * s + m] < blo[m]) blo[m] = X[3 * s + m];
            if (X[3 * s + m] > bhi[m]) bhi[m] = X[3 * s + m];
        }
    uint64_t* key = malloc(sizeof(uint64_t) * nF);
    for (int64_t s = 0; s < nF; ++s) {
        uint32_t code = (bh_spread10(bh_quant(X[3 * s], blo[0], bhi[0])) << 2) |
                        (bh_spread10(bh_quant(X[3 * s + 1], blo[1], bhi[1])) << 1) |
                        bh_spread10(bh_quant(X[3 * s + 2], blo[2], bhi[2]));
        key[s] = ((uint64_t)code << 32) | (uint64_t)s;
        T->order[s] = s;
    }
    bh_sort_keys = key;
    qsort(T->order, nF, sizeof(int64_t), bh_cmp);
    free(key);
    /* leaves */
    for (int64_t i = 0; i < M; ++i)
        for (int m = 0; m < 3; ++m) { T->lo[3 * i + m] = INFINITY; T->hi[3 * i + m] = -INFINITY; }
    double* sx = calloc(3 * M, sizeof(double));
    for (int64_t l = 0; l < T->P; ++l) {
        const int64_t node = T->P + l;
        for (int64_t p = l * leaf; p < (l + 1) * leaf && p < nF; ++p) {
            const int64_t s = T->order[p];
            T->a[node] += A[s];
            for (int m = 0; m < 3; ++m) {
                sx[3 * node + m] += A[s] * X[3 * s + m];
                if (T->flo[3 * s + m] < T->lo[3 * node + m]) T->lo[3 * node + m] = T->flo[3 * s + m];
                if (T->fhi[3 * s + m] > T->hi[3 * node + m]) T->hi[3 * node + m] = T->fhi[3 * s + m];
            }
        }
    }
    for (int64_t node = T->P - 1; node >= 1; --node) {
        const int64_t L = 2 * node, R = 2 * node + 1;
        T->a[node] = T->a[L] + T->a[R];
        for (int m = 0; m < 3; ++m) {
            sx[3 * node + m] = sx[3 * L + m] + sx[3 * R + m];
            T->lo[3 * node + m] = T->lo[3 * L + m] < T->lo[3 * R + m] ? T->lo[3 * L + m] : T->lo[3 * R + m];
            T->hi[3 * node + m] = T->hi[3 * L + m] > T->hi[3 * R + m] ? T->hi[3 * L + m] : T->hi[3 * R + m];
        }
    }
    for (int64_t node = 1; node < M; ++node) {
        if (!(T->a[node] > 0.0)) continue;
        double r2 = 0.0;
        for (int m = 0; m < 3; ++m) {
            T->X[3 * node + m] = sx[3 * node + m] / T->a[node];
            double u = T->X[3 * node + m] - T->lo[3 * node + m];
            double v = T->hi[3 * node + m] - T->X[3 * node + m];
            double w = u > v ? u : v;
            r2 += w * w;
        }
        T->r2[node] = r2;
    }
    free(sx);
}

static void bh_free(bh_tree* T)
{
    free(T->order); free(T->lo); free(T->hi); free(T->a); free(T->X); free(T->r2);
    free(T->flo); free(T->fhi); free(T->fr2);
}

static int bh_admissible(const bh_tree* T, int64_t s, int64_t node, double theta)
{
    double d2 = 0.0;
    for (int m = 0; m < 3; ++m) {
        double g1 = T->lo[3 * node + m] - T->fhi[3 * s + m];
        double g2 = T->flo[3 * s + m] - T->hi[3 * node + m];
        double g = g1 > g2 ? g1 : g2;
        if (g < 0.0) g = 0.0;
        d2 += g * g;
    }
    double r2 = T->fr2[s] > T->r2[node] ? T->fr2[s] : T->r2[node];
    return r2 < (theta * theta) * d2;
}

/* One face's interaction list, in traversal order: kinds[q] = 0 for a node, 1 for a face,
 * ids[q] its index.  Returns the count; the arrays are grown as needed. */
static int64_t bh_list(const bh_tree* T, int64_t s, double theta, int** kinds, int64_t** ids, int64_t* cap)
{
    int64_t n = 0;
    int64_t stack[128];
    int sp = 0;
    stack[sp++] = 1;
    while (sp > 0) {
        const int64_t node = stack[--sp];
        if (!(T->a[node] > 0.0)) continue;
        int leafnode = node >= T->P;
        if (n + T->leaf + 1 > *cap) {
            *cap = 2 * (*cap) + T->leaf + 1;
            *kinds = realloc(*kinds, sizeof(int) * (*cap));
            *ids = realloc(*ids, sizeof(int64_t) * (*cap));
        }
        if (bh_admissible(T, s, node, theta)) {
            (*kinds)[n] = 0; (*ids)[n] = node; ++n;
        } else if (leafnode) {
            const int64_t l = node - T->P;
            for (int64_t p = l * T->leaf; p < (l + 1) * T->leaf && p < T->nF; ++p) {
                const int64_t t = T->order[p];
                if (t == s) continue;
                (*kinds)[n] = 1; (*ids)[n] = t; ++n;
            }
        } else {
            stack[sp++] = 2 * node + 1;      /* right popped after left */
            stack[sp++] = 2 * node;
        }
    }
    return n;
}

/* E_BH and (optionally) its differential at vertices V, with the tree membership and the
 * interaction lists taken from vertices V0 (V0 = V for the plain evaluation; a different V
 * evaluates E_BH with the lists frozen, for finite differences).  counts[0] = far terms,
 * counts[1] = near terms (over all faces). */
EXPORT double tpo_bh_frozen(const double* V0, const double* V, int64_t nV, const int32_t* F, int64_t nF,
                            double alpha, double beta, double theta, int leaf, double* dE,
                            int64_t* counts)
{
    double* X0 = calloc(3 * nF, sizeof(double));
    double* N0 = calloc(3 * nF, sizeof(double));
    double* A0 = calloc(nF, sizeof(double));
    double* C0 = calloc(3 * nF, sizeof(double));
    all_faces(V0, F, nF, X0, N0, A0, C0);
    bh_tree T;
    bh_build(V0, F, nF, X0, A0, leaf, &T);
    /* quantities at V (same membership) */
    double* X = malloc(sizeof(double) * 3 * nF);
    double* N = malloc(sizeof(double) * 3 * nF);
    double* A = malloc(sizeof(double) * nF);
    double* C = malloc(sizeof(double) * 3 * nF);
    all_faces(V, F, nF, X, N, A, C);
    const int64_t M = 2 * T.P;
    double* na = calloc(M, sizeof(double));
    double* nX = calloc(3 * M, sizeof(double));
    {
        double* sx = calloc(3 * M, sizeof(double));
        for (int64_t l = 0; l < T.P; ++l)
            for (int64_t p = l * leaf; p < (l + 1) * leaf && p < nF; ++p) {
                const int64_t s = T.order[p];
                na[T.P + l] += A[s];
                for (int m = 0; m < 3; ++m) sx[3 * (T.P + l) + m] += A[s] * X[3 * s + m];
            }
        for (int64_t node = T.P - 1; node >= 1; --node) {
            na[node] = na[2 * node] + na[2 * node + 1];
            for (int m = 0; m < 3; ++m) sx[3 * node + m] = sx[3 * (2 * node) + m] + sx[3 * (2 * node + 1) + m];
        }
        for (int64_t node = 1; node < M; ++node)
            if (na[node] > 0.0)
                for (int m = 0; m < 3; ++m) nX[3 * node + m] = sx[3 * node + m] / na[node];
        free(sx);
    }
    double* gface = dE ? calloc(7 * nF, sizeof(double)) : NULL;
    double* gnode = dE ? calloc(4 * M, sizeof(double)) : NULL;
    int* kinds = NULL;
    int64_t* ids = NULL;
    int64_t cap = 0, nfar = 0, nnear = 0;
    double E = 0.0;
    for (int64_t s = 0; s < nF; ++s) {
        const int64_t n = bh_list(&T, s, theta, &kinds, &ids, &cap);
        double row = 0.0;
        for (int64_t q = 0; q < n; ++q) {
            const int far = kinds[q] == 0;
            const int64_t id = ids[q];
            const double* Y = far ? nX + 3 * id : X + 3 * id;
            const double w = far ? na[id] : A[id];
            far ? ++nfar : ++nnear;
            double dKdd[3], dKdN[3];
            const double K = tp_kernel_grad(X + 3 * s, N + 3 * s, Y, alpha, beta, dKdd, dKdN);
            row += K * A[s] * w;
            if (!dE) continue;
            double* gs = gface + 7 * s;
            for (int m = 0; m < 3; ++m) {
                gs[m] += A[s] * w * dKdd[m];
                gs[3 + m] += A[s] * w * dKdN[m];
            }
            gs[6] += w * K;
            if (far) {
                double* gn = gnode + 4 * id;
                for (int m = 0; m < 3; ++m) gn[m] -= A[s] * w * dKdd[m];
                gn[3] += A[s] * K;
            } else {
                double* gt = gface + 7 * id;
                for (int m = 0; m < 3; ++m) gt[m] -= A[s] * w * dKdd[m];
                gt[6] += A[s] * K;
            }
        }
        E += row;
    }
    if (dE) {
        /* node derivatives to member faces */
        for (int64_t l = 0; l < T.P; ++l)
            for (int64_t p = l * leaf; p < (l + 1) * leaf && p < nF; ++p) {
                const int64_t t = T.order[p];
                for (int64_t node = T.P + l; node >= 1; node /= 2) {
                    if (!(na[node] > 0.0)) continue;
                    const double* gn = gnode + 4 * node;
                    double proj = 0.0;
                    for (int m = 0; m < 3; ++m) {
                        gface[7 * t + m] += (A[t] / na[node]) * gn[m];
                        proj += (X[3 * t + m] - nX[3 * node + m]) * gn[m];
                    }
                    gface[7 * t + 6] += gn[3] + proj / na[node];
                }
            }
        tpo_face_to_vertex(V, nV, F, nF, gface, dE);
        free(gface); free(gnode);
    }
    if (counts) { counts[0] = nfar; counts[1] = nnear; }
    free(kinds); free(ids); free(na); free(nX);
    free(X0); free(N0); free(A0); free(C0); free(X); free(N); free(A); free(C);
    bh_free(&T);
    return E;
}

/* L^sigma u with the Barnes-Hut approximation of Sec. 4.1 carried over to the kernel
 * matrix of the fractional operator (Sec. 5.1.1), on the tree and interaction lists of
 * tpo_bh_frozen (same admissibility, same traversal).  For face S the exact row
 *   w(S) = a_S sum_{T != S} k(X_S, X_T) a_T (ubar_S - ubar_T),   k = |d|^-(2 sigma + 2),
 * takes, for an admissible node I, the kernel at the node's barycenter for all its faces:
 *   sum_{T in I} k(X_S, X_T) a_T (ubar_S - ubar_T)  ~  k(X_S, X_I) (a_I ubar_S - m_I),
 *   m_I = sum_{T in I} a_T ubar_T   (sums in sorted order, children left then right),
 * and a leaf that is not admissible adds its faces T != S exactly.  Then, as for the direct
 * sums, (L u)_i = 2 sum_{S ni i} w(S) / 3.  theta = 0 gives the direct sum.  k <= 64. */
EXPORT int tpo_bh_fractional(const double* V, int64_t nV, const int32_t* F, int64_t nF, double sigma,
                             double theta, int leaf, const double* u, int k, double* Lu)
{
    if (k < 1 || k > 64) return 1;
    double *X, *A, *ub;
    fractional_prepare(V, F, nF, u, k, &X, &A, &ub);
    bh_tree T;
    bh_build(V, F, nF, X, A, leaf, &T);
    const int64_t M = 2 * T.P;
    double* mI = calloc(M * k, sizeof(double));
    for (int64_t l = 0; l < T.P; ++l)
        for (int64_t p = l * leaf; p < (l + 1) * leaf && p < nF; ++p) {
            const int64_t t = T.order[p];
            for (int c = 0; c < k; ++c) mI[(T.P + l) * k + c] += A[t] * ub[t * k + c];
        }
    for (int64_t node = T.P - 1; node >= 1; --node)
        for (int c = 0; c < k; ++c) mI[node * k + c] = mI[2 * node * k + c] + mI[(2 * node + 1) * k + c];
    const double expo = -(2.0 * sigma + 2.0) * 0.5;
    double* w = calloc(nF * k, sizeof(double));
#pragma omp parallel
    {
        int* kinds = NULL;
        int64_t* ids = NULL;
        int64_t cap = 0;
        double acc[64];
#pragma omp for schedule(dynamic, 8)
        for (int64_t s = 0; s < nF; ++s) {
            const int64_t n = bh_list(&T, s, theta, &kinds, &ids, &cap);
            for (int c = 0; c < k; ++c) acc[c] = 0.0;
            for (int64_t q = 0; q < n; ++q) {
                const int far = kinds[q] == 0;
                const int64_t id = ids[q];
                const double* Y = far ? T.X + 3 * id : X + 3 * id;
                double d0 = X[3 * s] - Y[0], d1 = X[3 * s + 1] - Y[1], d2 = X[3 * s + 2] - Y[2];
                const double kv = pow(d0 * d0 + d1 * d1 + d2 * d2, expo);
                for (int c = 0; c < k; ++c)
                    acc[c] += far ? kv * (T.a[id] * ub[s * k + c] - mI[id * k + c])
                                  : kv * A[id] * (ub[s * k + c] - ub[id * k + c]);
            }
            for (int c = 0; c < k; ++c) w[s * k + c] = A[s] * acc[c];
        }
        free(kinds);
        free(ids);
    }
    tpo_fractional_gather(F, nF, nV, w, k, Lu);
    free(w); free(mI); free(X); free(A); free(ub);
    bh_free(&T);
    return 0;
}

/* Block cluster tree and hierarchical multiplication (Sec. 5.1.4, 5.1.5) for the kernel
 * matrix of the fractional operator, K_ST = (1 - delta_ST) k(X_S, X_T), k = |d|^-(2 sigma + 2).
 * Clusters are the nodes of the tree of tpo_bh_frozen.  Two clusters (I, J) are a separated
 * pair when max(r_I, r_J) < chi dist(I, J) (r: from the area-weighted barycenter to the
 * farthest corner of the cluster's box; dist: between the two boxes, which contain the
 * clusters' convex hulls -- reading: the same boxes as Barnes-Hut, strict inequality so that
 * chi = 0 separates nothing).  Starting from (root, root), a pair that is not separated and
 * not made of two leaves is split into the pairs of the children (all leaves lie at the
 * same depth).  Admissible blocks (separated) are rank one, 1_I k(X_I, X_J) 1_J^T;
 * inadmissible ones (two leaves, not separated) are exact.  With y = K~ x,
 *   w(S) = a_S (ubar_S (K~ a)(S) - (K~ (a ubar))(S)),
 * the kernel-matrix form of the fractional operator's row sums (Sec. 5.1.1), and
 * (L u)_i = 2 sum_{S ni i} w(S) / 3.  The products are taken block by block from the
 * definition (no upward / downward passes).  chi = 0 gives the direct sum.  k <= 64.
 * counts[0] = admissible blocks, counts[1] = inadmissible blocks. */
static double bct_sep(const bh_tree* T, int64_t I, int64_t J, double chi)
{
    double d2 = 0.0;
    for (int m = 0; m < 3; ++m) {
        double g1 = T->lo[3 * J + m] - T->hi[3 * I + m];
        double g2 = T->lo[3 * I + m] - T->hi[3 * J + m];
        double g = g1 > g2 ? g1 : g2;
        if (g < 0.0) g = 0.0;
        d2 += g * g;
    }
    double r2 = T->r2[I] > T->r2[J] ? T->r2[I] : T->r2[J];
    return r2 < (chi * chi) * d2;
}

EXPORT int tpo_bct_fractional(const double* V, int64_t nV, const int32_t* F, int64_t nF, double sigma,
                              double chi, int leaf, const double* u, int k, double* Lu, int64_t* counts)
{
    if (k < 1 || k > 63) return 1;
    double *X, *A, *ub;
    fractional_prepare(V, F, nF, u, k, &X, &A, &ub);
    bh_tree T;
    bh_build(V, F, nF, X, A, leaf, &T);
    const int kk = k + 1;                       /* x = [a, a ubar] */
    double* x = malloc(sizeof(double) * nF * kk);
    double* y = calloc(nF * kk, sizeof(double));
    for (int64_t t = 0; t < nF; ++t) {
        x[t * kk] = A[t];
        for (int c = 0; c < k; ++c) x[t * kk + 1 + c] = A[t] * ub[t * k + c];
    }
    const double expo = -(2.0 * sigma + 2.0) * 0.5;
    /* blocks by a breadth-first split of (root, root) */
    int64_t cap = 1024, n = 1, head = 0, nadm = 0, ninad = 0;
    int64_t* qI = malloc(sizeof(int64_t) * cap);
    int64_t* qJ = malloc(sizeof(int64_t) * cap);
    qI[0] = 1; qJ[0] = 1;
    double* xs = malloc(sizeof(double) * kk);
    while (head < n) {
        const int64_t I = qI[head], J = qJ[head];
        ++head;
        if (!(T.a[I] > 0.0) || !(T.a[J] > 0.0)) continue;
        const int64_t lI0 = I >= T.P ? (I - T.P) * leaf : 0, lJ0 = J >= T.P ? (J - T.P) * leaf : 0;
        if (bct_sep(&T, I, J, chi)) {
            ++nadm;
            /* y_S += k(X_I, X_J) sum_{T in J} x_T for S in I: faces of a cluster are the sorted
             * positions [first, last) of its subtree */
            int64_t depthI = 0, depthJ = 0, a = I, b = J;
            while (a < T.P) { a *= 2; ++depthI; }
            while (b < T.P) { b *= 2; ++depthJ; }
            const int64_t I0 = (a - T.P) * leaf, I1 = (a - T.P + ((int64_t)1 << depthI)) * leaf;
            const int64_t J0 = (b - T.P) * leaf, J1 = (b - T.P + ((int64_t)1 << depthJ)) * leaf;
            double d0 = T.X[3 * I] - T.X[3 * J], d1 = T.X[3 * I + 1] - T.X[3 * J + 1], d2 = T.X[3 * I + 2] - T.X[3 * J + 2];
            const double kv = pow(d0 * d0 + d1 * d1 + d2 * d2, expo);
            for (int c = 0; c < kk; ++c) xs[c] = 0.0;
            for (int64_t p = J0; p < J1 && p < nF; ++p)
                for (int c = 0; c < kk; ++c) xs[c] += x[T.order[p] * kk + c];
            for (int64_t p = I0; p < I1 && p < nF; ++p)
                for (int c = 0; c < kk; ++c) y[T.order[p] * kk + c] += kv * xs[c];
        } else if (I >= T.P) {          /* two leaves (same depth): exact block */
            ++ninad;
            for (int64_t p = lI0; p < lI0 + leaf && p < nF; ++p) {
                const int64_t S = T.order[p];
                for (int64_t q = lJ0; q < lJ0 + leaf && q < nF; ++q) {
                    const int64_t t = T.order[q];
                    if (t == S) continue;
                    double d0 = X[3 * S] - X[3 * t], d1 = X[3 * S + 1] - X[3 * t + 1], d2 = X[3 * S + 2] - X[3 * t + 2];
                    const double kv = pow(d0 * d0 + d1 * d1 + d2 * d2, expo);
                    for (int c = 0; c < kk; ++c) y[S * kk + c] += kv * x[t * kk + c];
                }
            }
        } else {
            if (n + 4 > cap) {
                cap *= 2;
                qI = realloc(qI, sizeof(int64_t) * cap);
                qJ = realloc(qJ, sizeof(int64_t) * cap);
            }
            for (int e = 0; e < 2; ++e)
                for (int f = 0; f < 2; ++f) { qI[n] = 2 * I + e; qJ[n] = 2 * J + f; ++n; }
        }
    }
    double* w = malloc(sizeof(double) * nF * k);
    for (int64_t S = 0; S < nF; ++S)
        for (int c = 0; c < k; ++c) w[S * k + c] = A[S] * (ub[S * k + c] * y[S * kk] - y[S * kk + 1 + c]);
    tpo_fractional_gather(F, nF, nV, w, k, Lu);
    if (counts) { counts[0] = nadm; counts[1] = ninad; }
    free(w); free(x); free(y); free(xs); free(qI); free(qJ); free(X); free(A); free(ub);
    bh_free(&T);
    return 0;
}

/* The sorted face order of the tree (for checks of the build). */
EXPORT void tpo_bh_order(const double* V, const int32_t* F, int64_t nF, int leaf, int64_t* order)
{
    double* X = malloc(sizeof(double) * 3 * nF);
    double* N = malloc(sizeof(double) * 3 * nF);
    double* A = malloc(sizeof(double) * nF);
    double* C = malloc(sizeof(double) * 3 * nF);
    all_faces(V, F, nF, X, N, A, C);
    bh_tree T;
    bh_build(V, F, nF, X, A, leaf, &T);
    memcpy(order, T.order, sizeof(int64_t) * nF);
    bh_free(&T);
    free(X); free(N); free(A); free(C);
}

/* Static obstacle potential by Barnes-Hut (Sec. 7.3.2, approximated as in Sec. 4.1).  The tree
 * of bh_build over the obstacle's faces.  The potential is evaluated at the barycenter X_T of a
 * surface face, a point without extent, so in the admissibility test of bh_admissible the
 * target radius is zero: node I is admissible when r_I^2 < theta^2 dist(X_T, box_I)^2, and then
 * contributes a_I |X_I - X_T|^-p; the faces of a leaf that is not admissible contribute one by
 * one.  Nodes are visited depth first, left child first.  The differential is the exact one of
 * this approximation with its lists held fixed; the obstacle does not move, so only the surface
 * side exists and the chain rule is that of tpo_obstacle.  counts: far terms, near terms. */
EXPORT double tpo_obstacle_bh(const double* V, int64_t nV, const int32_t* F, int64_t nF, const double* Vo,
                              const int32_t* Fo, int64_t nFo, double p, double theta, int leaf, double* dE,
                              int64_t* counts)
{
    double* XO = malloc(sizeof(double) * 3 * nFo);
    double* NO = malloc(sizeof(double) * 3 * nFo);
    double* AO = malloc(sizeof(double) * nFo);
    double* CO = malloc(sizeof(double) * 3 * nFo);
    all_faces(Vo, Fo, nFo, XO, NO, AO, CO);
    bh_tree T;
    bh_build(Vo, Fo, nFo, XO, AO, leaf, &T);
    if (dE) memset(dE, 0, sizeof(double) * 3 * nV);
    int64_t nfar = 0, nnear = 0;
    double E = 0.0;
    for (int64_t t = 0; t < nF; ++t) {
        double X[3], N[3], a, c[3];
        face_quantities(V, F, t, X, N, &a, c);
        double phi = 0.0, g[3] = {0.0, 0.0, 0.0};
        int64_t stack[128];
        int sp = 0;
        stack[sp++] = 1;
        while (sp > 0) {
            const int64_t node = stack[--sp];
            if (!(T.a[node] > 0.0)) continue;
            double d2 = 0.0;
            for (int m = 0; m < 3; ++m) {
                double g1 = T.lo[3 * node + m] - X[m], g2 = X[m] - T.hi[3 * node + m];
                double gm = g1 > g2 ? g1 : g2;
                if (gm < 0.0) gm = 0.0;
                d2 += gm * gm;
            }
            const double* Y = NULL;
            double w = 0.0;
            if (T.r2[node] < (theta * theta) * d2) {
                Y = T.X + 3 * node;
                w = T.a[node];
                ++nfar;
            } else if (node >= T.P) {
                const int64_t l = node - T.P;
                for (int64_t q = l * T.leaf; q < (l + 1) * T.leaf && q < nFo; ++q) {
                    const int64_t s = T.order[q];
                    double d[3] = {X[0] - XO[3 * s], X[1] - XO[3 * s + 1], X[2] - XO[3 * s + 2]};
                    double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
                    double ws = AO[s] * pow(r2, -0.5 * p);
                    phi += ws;
                    for (int m = 0; m < 3; ++m) g[m] += -p * ws / r2 * d[m];
                    ++nnear;
                }
                continue;
            } else {
                stack[sp++] = 2 * node + 1;
                stack[sp++] = 2 * node;
                continue;
            }
            double d[3] = {X[0] - Y[0], X[1] - Y[1], X[2] - Y[2]};
            double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
            double ws = w * pow(r2, -0.5 * p);
            phi += ws;
            for (int m = 0; m < 3; ++m) g[m] += -p * ws / r2 * d[m];
        }
        E += a * phi;
        if (!dE) continue;
        for (int corner = 0; corner < 3; ++corner) {
            const double* fj = V + 3 * (int64_t)F[3 * t + (corner + 1) % 3];
            const double* fk = V + 3 * (int64_t)F[3 * t + (corner + 2) % 3];
            double e[3] = {fk[0] - fj[0], fk[1] - fj[1], fk[2] - fj[2]};
            double da[3] = {0.5 * (N[1] * e[2] - N[2] * e[1]), 0.5 * (N[2] * e[0] - N[0] * e[2]),
                            0.5 * (N[0] * e[1] - N[1] * e[0])};
            int64_t i = F[3 * t + corner];
            for (int m = 0; m < 3; ++m) dE[3 * i + m] += a * g[m] / 3.0 + phi * da[m];
        }
    }
    if (counts) { counts[0] = nfar; counts[1] = nnear; }
    bh_free(&T);
    free(XO); free(NO); free(AO); free(CO);
    return E;
}
