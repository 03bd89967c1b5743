// Dynamic remeshing (Sec. 6): edge splits and collapses against a target length L0, then
// N rounds of Delaunay edge flips and tangential smoothing toward the face circumcenters.
//
// Topology editing is serial, branchy work on O(F) data that runs once between descent
// steps, so it runs on the host, in C++; the resident device state of a problem depends on
// the topology (incidence, sparsity pattern, preconditioner blocks, Morton order), so the
// caller creates a new problem from the remeshed arrays.
//
// Order of the operations (the paper gives the rules, not an order): each pass visits the
// edges as sorted vertex pairs (a < b) present at its start, tests an edge's current length
// when it is reached, and leaves edges created during the pass to the next pass.  A split
// numbers the new vertex next and puts it at the midpoint; a collapse keeps the smaller
// index at the midpoint and is refused when a remaining face around either end would flip
// its normal, or when the ends share a neighbour other than the two vertices opposite the
// edge (the link condition that keeps the surface a manifold).  The Delaunay condition of
// an interior edge is that its opposite angles sum to at most pi; a flip is refused when
// the new edge exists already; sweeps repeat until one flips nothing (at most 64).
// Smoothing moves every vertex by rho sum_S a_S (c_S - f_i) / sum_S a_S over its faces S
// (c_S the circumcenter), projected onto the plane of the area-weighted vertex normal;
// vertices on boundary edges stay.  Faces keep their orientation.  The edge-to-face lists
// are kept sorted by face number, so every choice depends on the mesh alone.
#include "tp_internal.h"

#include <algorithm>
#include <array>
#include <cmath>
#include <unordered_map>
#include <vector>

// Products and sums are rounded one by one (no fused multiply-adds), as written.
#pragma clang fp contract(off)

namespace tp {

namespace {

using Face = std::array<int32_t, 3>;

struct Remesher {
    std::vector<double> V;                                // 3 per vertex
    std::vector<Face> F;
    std::vector<char> fdead, valive;
    std::unordered_map<uint64_t, std::vector<int32_t>> ef;   // edge -> faces (ascending)
    std::vector<std::vector<int32_t>> vf;                 // vertex -> faces (live)

    static uint64_t key(int32_t a, int32_t b)
    {
        const uint32_t lo = (uint32_t)std::min(a, b), hi = (uint32_t)std::max(a, b);
        return ((uint64_t)lo << 32) | hi;
    }
    static void insert_sorted(std::vector<int32_t>& v, int32_t x)
    {
        v.insert(std::lower_bound(v.begin(), v.end(), x), x);
    }
    static void erase_one(std::vector<int32_t>& v, int32_t x)
    {
        auto it = std::find(v.begin(), v.end(), x);
        if (it != v.end()) v.erase(it);
    }
    void add_face(int32_t q)
    {
        const Face& f = F[q];
        for (int c = 0; c < 3; ++c) {
            insert_sorted(ef[key(f[c], f[(c + 1) % 3])], q);
            insert_sorted(vf[f[c]], q);
        }
    }
    void remove_face(int32_t q)
    {
        const Face& f = F[q];
        for (int c = 0; c < 3; ++c) {
            const uint64_t k = key(f[c], f[(c + 1) % 3]);
            auto it = ef.find(k);
            if (it != ef.end()) {
                erase_one(it->second, q);
                if (it->second.empty()) ef.erase(it);
            }
            erase_one(vf[f[c]], q);
        }
    }
    std::vector<uint64_t> sorted_edges() const
    {
        std::vector<uint64_t> e;
        e.reserve(ef.size());
        for (const auto& kv : ef) e.push_back(kv.first);
        std::sort(e.begin(), e.end());
        return e;
    }
    const double* P(int32_t v) const { return V.data() + 3 * (size_t)v; }
    double dist(int32_t a, int32_t b) const
    {
        const double dx = P(a)[0] - P(b)[0], dy = P(a)[1] - P(b)[1], dz = P(a)[2] - P(b)[2];
        return std::sqrt(dx * dx + dy * dy + dz * dz);
    }
    static void cross(const double* u, const double* w, double* n)
    {
        n[0] = u[1] * w[2] - u[2] * w[1];
        n[1] = u[2] * w[0] - u[0] * w[2];
        n[2] = u[0] * w[1] - u[1] * w[0];
    }
    // (f1 - f0) x (f2 - f0) with positions p0, p1, p2
    static void normal3(const double* p0, const double* p1, const double* p2, double* n)
    {
        const double u[3] = {p1[0] - p0[0], p1[1] - p0[1], p1[2] - p0[2]};
        const double w[3] = {p2[0] - p0[0], p2[1] - p0[1], p2[2] - p0[2]};
        cross(u, w, n);
    }

    void split_pass(double L0)
    {
        for (uint64_t k : sorted_edges()) {
            auto it = ef.find(k);
            if (it == ef.end()) continue;
            const int32_t a = (int32_t)(k >> 32), b = (int32_t)(k & 0xffffffffu);
            if (!(dist(a, b) > 1.5 * L0)) continue;
            const int32_t m = (int32_t)(V.size() / 3);
            for (int c = 0; c < 3; ++c) V.push_back(0.5 * (P(a)[c] + P(b)[c]));
            valive.push_back(1);
            vf.emplace_back();
            const std::vector<int32_t> faces = it->second;      // a copy: the lists change below
            for (int32_t q : faces) {
                const Face f = F[q];
                int c0 = 0;
                while (f[c0] == a || f[c0] == b) ++c0;
                const int32_t x = f[c0], y = f[(c0 + 1) % 3], z = f[(c0 + 2) % 3];
                remove_face(q);
                F[q] = {x, y, m};
                add_face(q);
                const int32_t r = (int32_t)F.size();
                F.push_back({x, m, z});
                fdead.push_back(0);
                add_face(r);
            }
        }
    }

    bool collapse_ok(int32_t a, int32_t b, const std::vector<int32_t>& edge_faces) const
    {
        std::vector<int32_t> na, nb, opp;
        for (int32_t q : vf[a])
            for (int32_t v : F[q])
                if (v != a) na.push_back(v);
        for (int32_t q : vf[b])
            for (int32_t v : F[q])
                if (v != b) nb.push_back(v);
        for (int32_t q : edge_faces)
            for (int32_t v : F[q])
                if (v != a && v != b) opp.push_back(v);
        for (auto* s : {&na, &nb, &opp}) {
            std::sort(s->begin(), s->end());
            s->erase(std::unique(s->begin(), s->end()), s->end());
        }
        std::vector<int32_t> common;
        std::set_intersection(na.begin(), na.end(), nb.begin(), nb.end(), std::back_inserter(common));
        if (common != opp) return false;
        const double mid[3] = {0.5 * (P(a)[0] + P(b)[0]), 0.5 * (P(a)[1] + P(b)[1]), 0.5 * (P(a)[2] + P(b)[2])};
        for (int32_t end : {a, b})
            for (int32_t q : vf[end]) {
                if (std::find(edge_faces.begin(), edge_faces.end(), q) != edge_faces.end()) continue;
                const Face& f = F[q];
                double n0[3], n1[3];
                normal3(P(f[0]), P(f[1]), P(f[2]), n0);
                const double* p[3];
                for (int c = 0; c < 3; ++c) p[c] = (f[c] == a || f[c] == b) ? mid : P(f[c]);
                normal3(p[0], p[1], p[2], n1);
                if (!(n0[0] * n1[0] + n0[1] * n1[1] + n0[2] * n1[2] > 0.0)) return false;
            }
        return true;
    }

    void collapse_pass(double L0)
    {
        for (uint64_t k : sorted_edges()) {
            auto it = ef.find(k);
            if (it == ef.end()) continue;
            const int32_t a = (int32_t)(k >> 32), b = (int32_t)(k & 0xffffffffu);
            if (!valive[a] || !valive[b]) continue;
            if (!(dist(a, b) < 0.5 * L0)) continue;
            const std::vector<int32_t> edge_faces = it->second;
            if (!collapse_ok(a, b, edge_faces)) continue;
            for (int c = 0; c < 3; ++c) V[3 * (size_t)a + c] = 0.5 * (P(a)[c] + P(b)[c]);
            for (int32_t q : edge_faces) {
                remove_face(q);
                fdead[q] = 1;
            }
            const std::vector<int32_t> fb = vf[b];
            for (int32_t q : fb) {
                remove_face(q);
                for (int c = 0; c < 3; ++c)
                    if (F[q][c] == b) F[q][c] = a;
                add_face(q);
            }
            valive[b] = 0;
        }
    }

    static double angle_at(const double* p, const double* q, const double* r)
    {
        const double u[3] = {q[0] - p[0], q[1] - p[1], q[2] - p[2]};
        const double w[3] = {r[0] - p[0], r[1] - p[1], r[2] - p[2]};
        double n[3];
        cross(u, w, n);
        return std::atan2(std::sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]), u[0] * w[0] + u[1] * w[1] + u[2] * w[2]);
    }

    int64_t flip_pass(int max_sweeps)
    {
        int64_t total = 0;
        for (int sweep = 0; sweep < max_sweeps; ++sweep) {
            int64_t changed = 0;
            for (uint64_t k : sorted_edges()) {
                auto it = ef.find(k);
                if (it == ef.end() || it->second.size() != 2) continue;
                const int32_t a = (int32_t)(k >> 32), b = (int32_t)(k & 0xffffffffu);
                const int32_t q1 = it->second[0], q2 = it->second[1];
                const Face f1 = F[q1], f2 = F[q2];
                int32_t c = -1, d = -1;
                for (int t = 0; t < 3; ++t) {
                    if (f1[t] != a && f1[t] != b) c = f1[t];
                    if (f2[t] != a && f2[t] != b) d = f2[t];
                }
                if (c == d || ef.count(key(c, d))) continue;
                if (!(angle_at(P(c), P(a), P(b)) + angle_at(P(d), P(a), P(b)) > M_PI)) continue;
                int kc = 0;
                while (f1[kc] != c) ++kc;
                const int32_t p = f1[(kc + 1) % 3], q = f1[(kc + 2) % 3];
                remove_face(q1);
                remove_face(q2);
                F[q1] = {c, p, d};
                F[q2] = {d, q, c};
                add_face(q1);
                add_face(q2);
                ++changed;
            }
            total += changed;
            if (changed == 0) break;
        }
        return total;
    }

    static void circumcenter(const double* a, const double* b, const double* c, double* out)
    {
        const double u[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
        const double w[3] = {c[0] - a[0], c[1] - a[1], c[2] - a[2]};
        double n[3], nu[3], wn[3];
        cross(u, w, n);
        cross(n, u, nu);
        cross(w, n, wn);
        const double ww = w[0] * w[0] + w[1] * w[1] + w[2] * w[2];
        const double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
        const double nn = n[0] * n[0] + n[1] * n[1] + n[2] * n[2];
        for (int m = 0; m < 3; ++m) out[m] = a[m] + (nu[m] * ww + wn[m] * uu) / (2.0 * nn);
    }

    void smooth(double rho)
    {
        const size_t nV = V.size() / 3;
        std::vector<double> num(3 * nV, 0.0), den(nV, 0.0), nrm(3 * nV, 0.0);
        std::vector<char> fixed(nV, 0);
        for (const auto& kv : ef)
            if (kv.second.size() != 2) {
                fixed[kv.first >> 32] = 1;
                fixed[kv.first & 0xffffffffu] = 1;
            }
        for (size_t q = 0; q < F.size(); ++q) {
            if (fdead[q]) continue;
            const Face& f = F[q];
            double n[3], cc[3];
            normal3(P(f[0]), P(f[1]), P(f[2]), n);
            const double area = 0.5 * std::sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
            circumcenter(P(f[0]), P(f[1]), P(f[2]), cc);
            for (int32_t v : f) {
                for (int m = 0; m < 3; ++m) {
                    num[3 * v + m] += area * (cc[m] - P(v)[m]);
                    nrm[3 * v + m] += 0.5 * n[m];
                }
                den[v] += area;
            }
        }
        std::vector<double> out = V;
        for (size_t v = 0; v < nV; ++v) {
            if (!valive[v] || den[v] == 0.0 || fixed[v]) continue;
            double u[3], N[3];
            for (int m = 0; m < 3; ++m) u[m] = rho * num[3 * v + m] / den[v];
            const double nn = std::sqrt(nrm[3 * v] * nrm[3 * v] + nrm[3 * v + 1] * nrm[3 * v + 1] +
                                        nrm[3 * v + 2] * nrm[3 * v + 2]);
            for (int m = 0; m < 3; ++m) N[m] = nrm[3 * v + m] / nn;
            const double un = u[0] * N[0] + u[1] * N[1] + u[2] * N[2];
            for (int m = 0; m < 3; ++m) out[3 * v + m] = P((int32_t)v)[m] + (u[m] - un * N[m]);
        }
        V.swap(out);
    }
};

}  // namespace

}  // namespace tp

extern "C" tp_status tp_remesh(const double* V, int64_t nV, const int32_t* F, int64_t nF, double L0, int iterations,
                               double rho, double* V_out, int64_t cap_V, int32_t* F_out, int64_t cap_F,
                               int64_t* nV_out, int64_t* nF_out)
{
    using namespace tp;
    set_error("");
    if (!V || !F || !nV_out || !nF_out) { set_error("NULL argument"); return TP_E_INVALID_ARGUMENT; }
    if (nV < 3 || nF < 1 || nV > (int64_t)INT32_MAX / 4 || nF > (int64_t)INT32_MAX / 4) {
        set_error("need nV >= 3, nF >= 1 (and below 2^29)");
        return TP_E_INVALID_ARGUMENT;
    }
    if (!(L0 > 0.0) || !std::isfinite(L0) || iterations < 0 || !(rho >= 0.0 && rho < 1.0)) {
        set_error("need L0 > 0, iterations >= 0 and 0 <= rho < 1");
        return TP_E_INVALID_ARGUMENT;
    }
    Remesher R;
    R.V.assign(V, V + 3 * nV);
    for (int64_t v = 0; v < 3 * nV; ++v)
        if (!std::isfinite(V[v])) { set_error("non-finite vertex coordinates"); return TP_E_NONFINITE; }
    R.F.resize(nF);
    for (int64_t q = 0; q < nF; ++q)
        for (int c = 0; c < 3; ++c) {
            const int32_t i = F[3 * q + c];
            if (i < 0 || i >= nV) { set_error("a face refers to a vertex index outside [0, nV)"); return TP_E_BAD_INDEX; }
            R.F[q][c] = i;
        }
    R.fdead.assign(nF, 0);
    R.valive.assign(nV, 1);
    R.vf.assign(nV, {});
    for (int64_t q = 0; q < nF; ++q) R.add_face((int32_t)q);
    R.split_pass(L0);
    R.collapse_pass(L0);
    for (int it = 0; it < iterations; ++it) {
        R.flip_pass(64);
        R.smooth(rho);
    }
    // compaction: surviving vertices and faces in order
    const int64_t nv_all = (int64_t)(R.V.size() / 3);
    std::vector<int32_t> remap(nv_all, -1);
    int64_t nv = 0, nf = 0;
    for (int64_t v = 0; v < nv_all; ++v)
        if (R.valive[v]) remap[v] = (int32_t)nv++;
    for (size_t q = 0; q < R.F.size(); ++q)
        if (!R.fdead[q]) ++nf;
    *nV_out = nv;
    *nF_out = nf;
    if (!V_out || !F_out || nv > cap_V || nf > cap_F) {
        set_error("output arrays too small: need " + std::to_string(nv) + " vertices and " + std::to_string(nf) +
                  " faces (reported in nV_out, nF_out)");
        return TP_E_INVALID_ARGUMENT;
    }
    for (int64_t v = 0; v < nv_all; ++v)
        if (remap[v] >= 0)
            for (int c = 0; c < 3; ++c) V_out[3 * (int64_t)remap[v] + c] = R.V[3 * (size_t)v + c];
    int64_t o = 0;
    for (size_t q = 0; q < R.F.size(); ++q)
        if (!R.fdead[q]) {
            for (int c = 0; c < 3; ++c) F_out[3 * o + c] = remap[R.F[q][c]];
            ++o;
        }
    return TP_OK;
}
