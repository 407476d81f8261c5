// Per-element geometry and face connectivity in FP64 (host).
//
// Affine element maps (section "Implementation Aspects": Psi = A_k (r,s)^T +
// b_k, |A_k| the volume Jacobian, A_k^{-1} the factors of eq.
// dg-diff-local-to-global), outward unit normals, surface Jacobians
// (edge length / 2 in 2D, face area / 2 in 3D) and Fscale = sJ / J.
// Faces are matched combinatorially: equal sorted vertex tuples, the partner
// face's node order expressed as one of the face's vertex permutations.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <limits>
#include <stdexcept>
#include <unordered_map>

#include "host.hpp"

namespace dgw {

namespace {

struct FaceKey {
    std::array<int64_t, 3> v;
    bool operator==(const FaceKey &o) const { return v == o.v; }
};
struct FaceKeyHash {
    size_t operator()(const FaceKey &k) const {
        uint64_t h = 1469598103934665603ull;
        for (int64_t x : k.v) {
            h ^= (uint64_t)x + 0x9e3779b97f4a7c15ull + (h << 6) + (h >> 2);
            h *= 1099511628211ull;
        }
        return (size_t)h;
    }
};

[[noreturn]] void mesh_fail(int code, const std::string &m) { throw MeshError{code, m}; }

}  // namespace

Geometry build_geometry(const RefElement &ref, int dim, int64_t n_verts, const double *vx, const double *vy,
                        const double *vz, int64_t K, const int32_t *ev, const double *eps, const double *mu) {
    Geometry g;
    g.dim = dim;
    g.K = K;
    const int nv = dim + 1, Nf = ref.Nfaces, Np = ref.Np, fv = dim;
    g.J.resize(K);
    g.drst.resize((size_t)K * dim * dim);
    g.normal.resize((size_t)K * Nf * dim);
    g.sJ.resize((size_t)K * Nf);
    g.x.resize((size_t)K * Np);
    g.y.resize((size_t)K * Np);
    if (dim == 3) g.z.resize((size_t)K * Np);
    g.inradius.resize(K);
    g.eps.assign(K, 1.0);
    g.mu.assign(K, 1.0);
    for (int64_t k = 0; k < K; ++k) {
        if (eps) g.eps[k] = eps[k];
        if (mu) g.mu[k] = mu[k];
        if (!(g.eps[k] > 0.0) || !(g.mu[k] > 0.0) || !std::isfinite(g.eps[k]) || !std::isfinite(g.mu[k]))
            mesh_fail(-1, "eps and mu must be positive and finite");
    }
    for (int64_t k = 0; k < K; ++k) {
        double P[4][3] = {};
        for (int v = 0; v < nv; ++v) {
            const int64_t id = ev[k * nv + v];
            if (id < 0 || id >= n_verts) mesh_fail(-2, "vertex id out of range in element " + std::to_string(k));
            P[v][0] = vx[id];
            P[v][1] = vy[id];
            P[v][2] = dim == 3 ? vz[id] : 0.0;
        }
        // A = [dx/dr dx/ds (dx/dt); ...]: columns (P_i - P_0)/2
        double A[3][3] = {};
        for (int c = 0; c < dim; ++c)
            for (int rrow = 0; rrow < dim; ++rrow) A[rrow][c] = 0.5 * (P[c + 1][rrow] - P[0][rrow]);
        double J;
        double *G = &g.drst[(size_t)k * dim * dim];
        if (dim == 2) {
            J = A[0][0] * A[1][1] - A[0][1] * A[1][0];
            if (!(J > 0.0)) mesh_fail(-2, "element " + std::to_string(k) + " has non-positive Jacobian");
            G[0] = A[1][1] / J;   // r_x
            G[1] = -A[0][1] / J;  // r_y
            G[2] = -A[1][0] / J;  // s_x
            G[3] = A[0][0] / J;   // s_y
        } else {
            J = A[0][0] * (A[1][1] * A[2][2] - A[1][2] * A[2][1]) - A[0][1] * (A[1][0] * A[2][2] - A[1][2] * A[2][0]) +
                A[0][2] * (A[1][0] * A[2][1] - A[1][1] * A[2][0]);
            if (!(J > 0.0)) mesh_fail(-2, "element " + std::to_string(k) + " has non-positive Jacobian");
            // inverse via cofactors: rows are grad r, grad s, grad t
            G[0] = (A[1][1] * A[2][2] - A[1][2] * A[2][1]) / J;
            G[1] = (A[0][2] * A[2][1] - A[0][1] * A[2][2]) / J;
            G[2] = (A[0][1] * A[1][2] - A[0][2] * A[1][1]) / J;
            G[3] = (A[1][2] * A[2][0] - A[1][0] * A[2][2]) / J;
            G[4] = (A[0][0] * A[2][2] - A[0][2] * A[2][0]) / J;
            G[5] = (A[0][2] * A[1][0] - A[0][0] * A[1][2]) / J;
            G[6] = (A[1][0] * A[2][1] - A[1][1] * A[2][0]) / J;
            G[7] = (A[0][1] * A[2][0] - A[0][0] * A[2][1]) / J;
            G[8] = (A[0][0] * A[1][1] - A[0][1] * A[1][0]) / J;
        }
        g.J[k] = J;
        double area_sum = 0.0;
        for (int f = 0; f < Nf; ++f) {
            const int *vf = &ref.face_verts[f * fv];
            double n[3] = {0, 0, 0}, sj;
            if (dim == 2) {
                const double dx = P[vf[1]][0] - P[vf[0]][0], dy = P[vf[1]][1] - P[vf[0]][1];
                const double L = std::hypot(dx, dy);
                n[0] = dy / L;
                n[1] = -dx / L;
                sj = 0.5 * L;
            } else {
                double e1[3], e2[3];
                for (int c = 0; c < 3; ++c) {
                    e1[c] = P[vf[1]][c] - P[vf[0]][c];
                    e2[c] = P[vf[2]][c] - P[vf[0]][c];
                }
                n[0] = e1[1] * e2[2] - e1[2] * e2[1];
                n[1] = e1[2] * e2[0] - e1[0] * e2[2];
                n[2] = e1[0] * e2[1] - e1[1] * e2[0];
                int opp = 0;
                for (int v = 0; v < 4; ++v)
                    if (v != vf[0] && v != vf[1] && v != vf[2]) opp = v;
                double into = 0;
                for (int c = 0; c < 3; ++c) into += n[c] * (P[opp][c] - P[vf[0]][c]);
                const double nn = std::sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
                const double sgn = into > 0 ? -1.0 : 1.0;
                for (int c = 0; c < 3; ++c) n[c] *= sgn / nn;
                sj = 0.25 * nn;  // (area = |cross|/2) / (reference face area 2)
            }
            for (int c = 0; c < dim; ++c) g.normal[((size_t)k * Nf + f) * dim + c] = n[c];
            g.sJ[(size_t)k * Nf + f] = sj;
            area_sum += 2.0 * sj;
        }
        g.inradius[k] = dim == 2 ? 2.0 * (2.0 * J) / area_sum : 3.0 * (4.0 / 3.0 * J) / area_sum;
        // node coordinates from the barycentric weights of the reference nodes
        for (int n = 0; n < Np; ++n) {
            double lam[4];
            lam[1] = 0.5 * (1 + ref.r[n]);
            lam[2] = 0.5 * (1 + ref.s[n]);
            lam[3] = dim == 3 ? 0.5 * (1 + ref.t[n]) : 0.0;
            lam[0] = 1.0 - lam[1] - lam[2] - lam[3];
            double X[3] = {0, 0, 0};
            for (int v = 0; v < nv; ++v)
                for (int c = 0; c < 3; ++c) X[c] += lam[v] * P[v][c];
            g.x[(size_t)k * Np + n] = X[0];
            g.y[(size_t)k * Np + n] = X[1];
            if (dim == 3) g.z[(size_t)k * Np + n] = X[2];
        }
    }

    // Face matching.
    g.nbr_elem.assign((size_t)K * Nf, -1);
    g.nbr_face.assign((size_t)K * Nf, -1);
    g.nbr_orient.assign((size_t)K * Nf, 0);
    std::unordered_map<FaceKey, int64_t, FaceKeyHash> first;
    first.reserve((size_t)(K * Nf / 2 + 16));
    auto gvert = [&](int64_t k, int f, int q) -> int64_t { return ev[k * nv + ref.face_verts[f * fv + q]]; };
    for (int64_t k = 0; k < K; ++k)
        for (int f = 0; f < Nf; ++f) {
            FaceKey key{{-1, -1, -1}};
            for (int q = 0; q < fv; ++q) key.v[q] = gvert(k, f, q);
            std::sort(key.v.begin(), key.v.begin() + fv);
            for (int q = 1; q < fv; ++q)
                if (key.v[q] == key.v[q - 1]) mesh_fail(-2, "degenerate face in element " + std::to_string(k));
            auto it = first.find(key);
            const int64_t me = k * Nf + f;
            if (it == first.end()) {
                first.emplace(key, me);
                continue;
            }
            const int64_t other = it->second;
            if (other < 0) mesh_fail(-2, "non-conforming mesh: a face is shared by more than two elements");
            const int64_t k2 = other / Nf;
            const int f2 = int(other % Nf);
            it->second = -1;  // consumed
            // orientation of the partner's face relative to ours, both ways
            for (int side = 0; side < 2; ++side) {
                const int64_t ka = side == 0 ? k : k2, kb = side == 0 ? k2 : k;
                const int fa = side == 0 ? f : f2, fb = side == 0 ? f2 : f;
                std::array<int, 3> pi{0, 1, 2};
                for (int q = 0; q < fv; ++q) {
                    const int64_t gq = gvert(kb, fb, q);
                    int hit = -1;
                    for (int p = 0; p < fv; ++p)
                        if (gvert(ka, fa, p) == gq) hit = p;
                    if (hit < 0) mesh_fail(-2, "face vertex mismatch");
                    pi[q] = hit;
                }
                int o;
                if (dim == 2) {
                    o = pi[0] == 0 ? 0 : 1;
                } else {
                    static const int perms[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
                    o = -1;
                    for (int p = 0; p < 6; ++p)
                        if (perms[p][0] == pi[0] && perms[p][1] == pi[1] && perms[p][2] == pi[2]) o = p;
                }
                g.nbr_elem[(size_t)ka * Nf + fa] = kb;
                g.nbr_face[(size_t)ka * Nf + fa] = fb;
                g.nbr_orient[(size_t)ka * Nf + fa] = o;
            }
        }
    return g;
}

std::vector<int64_t> morton_order(const Geometry &g) {
    const int64_t K = g.K;
    const int dim = g.dim;
    const int Np = (int)(g.x.size() / std::max<int64_t>(K, 1));
    std::vector<double> c((size_t)K * dim);
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (int64_t k = 0; k < K; ++k) {
        for (int d = 0; d < dim; ++d) {
            const std::vector<double> &X = d == 0 ? g.x : d == 1 ? g.y : g.z;
            double s = 0;
            for (int n = 0; n < Np; ++n) s += X[(size_t)k * Np + n];
            s /= Np;
            c[(size_t)k * dim + d] = s;
            lo[d] = std::min(lo[d], s);
            hi[d] = std::max(hi[d], s);
        }
    }
    const int bits = dim == 2 ? 16 : 10;
    const double scale = double((1u << bits) - 1);
    std::vector<std::pair<uint64_t, int64_t>> key((size_t)K);
    for (int64_t k = 0; k < K; ++k) {
        uint64_t code = 0;
        uint32_t q[3] = {0, 0, 0};
        for (int d = 0; d < dim; ++d) {
            const double span = hi[d] > lo[d] ? hi[d] - lo[d] : 1.0;
            q[d] = (uint32_t)std::lround((c[(size_t)k * dim + d] - lo[d]) / span * scale);
        }
        for (int b = bits - 1; b >= 0; --b)
            for (int d = dim - 1; d >= 0; --d) code = (code << 1) | ((q[d] >> b) & 1u);
        key[k] = {code, k};
    }
    std::stable_sort(key.begin(), key.end());
    std::vector<int64_t> order((size_t)K);
    for (int64_t i = 0; i < K; ++i) order[i] = key[i].second;
    return order;
}

double cfl_dt(const RefElement &ref, const Geometry &g, double cfl_factor) {
    const std::vector<double> x = lgl_points(ref.N);
    double m = std::numeric_limits<double>::infinity();
    for (int64_t k = 0; k < g.K; ++k) m = std::min(m, g.inradius[k] * std::sqrt(g.eps[k] * g.mu[k]));
    return cfl_factor * 0.5 * (x[1] - x[0]) * m;
}

}  // namespace dgw
