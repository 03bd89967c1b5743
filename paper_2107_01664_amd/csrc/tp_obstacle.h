// Static obstacle potential (Sec. 7.3.2): a fixed mesh O repels the surface with
//   E_obs = sum_T a_T sum_{S in O} a_O(S) |X_O(S) - X_T|^-p,
// the potential of every face T of the surface evaluated at its barycenter and integrated
// over its area.
#pragma once
#include "tp_internal.h"

namespace tp {

// Obstacle face data: (X_O, a_O) in FP64 for cap_o entries (padding: zero area, far away).
int64_t obstacle_capacity(int64_t nFo);
hipError_t launch_obstacle_faces(const double* Vo, const int32_t* Fo, int64_t nFo, int64_t cap_o, double4* xo,
                                 hipStream_t s);
// Per surface face T (dx: the surface's FP64 face data, nF faces): e[T] = a_T phi(T) and the
// face partials of E_obs for the vertex chain rule, g = [7][gs]: dE/dX_T (3 rows), dE/dN_T = 0
// (3 rows), dE/da_T = phi(T) (1 row).
hipError_t launch_obstacle_pairs(const double4* dx, int64_t nF, const double4* xo, int64_t cap_o, double p,
                                 double* e, double* g, int64_t gs, hipStream_t s);

// The same potential and partials with Barnes-Hut over the obstacle (params.theta > 0): tree
// = launch_bh_build over the obstacle faces (xo their face data, unpadded order), counts[2] =
// far and near terms of this evaluation (cleared here).
hipError_t launch_obstacle_bh(const double4* dx, int64_t nF, const double4* xo, const BhBuffers& tree, int64_t nFo,
                              int leaf, double theta, double p, double* e, double* g, int64_t gs,
                              unsigned long long* counts, hipStream_t s);

// Implicit obstacles and attractors (Sec. 7.3.3) on analytic signed distances: kind 0 a plane,
// d(x) = n . x - c (q = n, c), kind 1 a sphere, d(x) = |x - q| - c.  The potential of one
// primitive is d^-p (obstacle) or |d|^p (attractor), weighted, evaluated at the face
// barycenters and integrated with the face areas.
constexpr int kMaxImplicit = 8;
struct ImplicitSet {
    int n = 0;
    int kind[kMaxImplicit];
    int attract[kMaxImplicit];
    double q[kMaxImplicit][3];
    double c[kMaxImplicit];
    double p[kMaxImplicit];
    double w[kMaxImplicit];
};
// Per surface face: e[T] = a_T sum_k w_k phi_k(X_T) and the face partials g = [7][gs] as for
// launch_obstacle_pairs.
hipError_t launch_implicit(const double4* dx, int64_t nF, const ImplicitSet& set, double* e, double* g, int64_t gs,
                           hipStream_t s);

// Vertex areas a(v) = sum of a_S / 3 over the faces S around v (dx: FP64 face data).
hipError_t launch_vertex_area(int64_t nV, const int32_t* vf_off, const int32_t* vf_idx, const double4* dx,
                              double* out, hipStream_t s);
// x[v] += t[label[v]] (n x 3 rows, t ncomp x 3).
hipError_t launch_add_translation(double* x, const int32_t* label, const double* t, int64_t n, hipStream_t s);

}  // namespace tp
