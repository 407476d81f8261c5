// Reference simplex of order N, built in FP64 on the host.
//
// The nodal basis is the Lagrange basis on Warburton's warp & blend points
// (the stability-optimised interpolation points the paper cites); M and the
// differentiation matrices come from an orthonormal (Koornwinder-Dubiner)
// simplex basis (section "Implementation Aspects"): with V the generalised
// Vandermonde matrix and V_r its r-derivative, D_r = V_r V^{-1},
// M = V^{-T} V^{-1}; LIFT = M^{-1} M^{dI} with M^{dI} the combined face mass
// matrix of eq. dg-lift (each face's mass matrix in its own reference
// coordinates, face parameter length 2 in 2D, reference face area 2 in 3D).
#include "host.hpp"

#include <algorithm>
#include <array>
#include <cmath>
#include <stdexcept>

namespace dgw {

// ---------------------------------------------------------------- linear algebra

Mat matmul(const Mat &A, const Mat &B) {
    Mat C(A.rows, B.cols);
    for (int i = 0; i < A.rows; ++i)
        for (int k = 0; k < A.cols; ++k) {
            const double a = A(i, k);
            if (a == 0.0) continue;
            for (int j = 0; j < B.cols; ++j) C(i, j) += a * B(k, j);
        }
    return C;
}

Mat transpose(const Mat &A) {
    Mat T(A.cols, A.rows);
    for (int i = 0; i < A.rows; ++i)
        for (int j = 0; j < A.cols; ++j) T(j, i) = A(i, j);
    return T;
}

Mat inverse(const Mat &A) {
    const int n = A.rows;
    Mat W(n, 2 * n);
    for (int i = 0; i < n; ++i) {
        for (int j = 0; j < n; ++j) W(i, j) = A(i, j);
        W(i, n + i) = 1.0;
    }
    for (int c = 0; c < n; ++c) {
        int p = c;
        for (int i = c + 1; i < n; ++i)
            if (std::fabs(W(i, c)) > std::fabs(W(p, c))) p = i;
        if (W(p, c) == 0.0) throw std::runtime_error("singular matrix");
        if (p != c)
            for (int j = 0; j < 2 * n; ++j) std::swap(W(p, j), W(c, j));
        const double inv = 1.0 / W(c, c);
        for (int j = 0; j < 2 * n; ++j) W(c, j) *= inv;
        for (int i = 0; i < n; ++i) {
            if (i == c) continue;
            const double f = W(i, c);
            if (f == 0.0) continue;
            for (int j = 0; j < 2 * n; ++j) W(i, j) -= f * W(c, j);
        }
    }
    Mat R(n, n);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) R(i, j) = W(i, n + j);
    return R;
}

// ---------------------------------------------------------------- 1D polynomials

// Orthonormal Jacobi polynomials P_0..P_nmax (weight (1-x)^a (1+x)^b) at x,
// by the three-term recurrence of the orthonormal family.
static void jacobi_all(double x, double a, double b, int nmax, double *p) {
    p[0] = std::sqrt(std::exp(std::lgamma(a + b + 2) - std::lgamma(a + 1) - std::lgamma(b + 1)) /
                     std::pow(2.0, a + b + 1));
    if (nmax == 0) return;
    p[1] = p[0] * (0.5 * (a + b + 2) * x + 0.5 * (a - b)) * std::sqrt((a + b + 3) / ((a + 1) * (b + 1)));
    double a_n = 2.0 / (2 + a + b) * std::sqrt((a + 1) * (b + 1) / (a + b + 3));
    for (int n = 1; n < nmax; ++n) {
        const double h = 2.0 * n + a + b;
        const double a_next = 2.0 / (h + 2) *
                              std::sqrt((n + 1) * (n + 1 + a + b) * (n + 1 + a) * (n + 1 + b) / ((h + 1) * (h + 3)));
        const double b_n = -(a * a - b * b) / (h * (h + 2));
        p[n + 1] = ((x - b_n) * p[n] - a_n * p[n - 1]) / a_next;
        a_n = a_next;
    }
}

static double jacobi(double x, double a, double b, int n) {
    double p[32];
    jacobi_all(x, a, b, n, p);
    return p[n];
}

// d/dx of the orthonormal P_n^(a,b) = sqrt(n (n+a+b+1)) P_{n-1}^(a+1,b+1).
static double jacobi_dx(double x, double a, double b, int n) {
    if (n == 0) return 0.0;
    return std::sqrt(n * (n + a + b + 1)) * jacobi(x, a + 1, b + 1, n - 1);
}

std::vector<double> lgl_points(int N) {
    std::vector<double> x(N + 1);
    x[0] = -1.0;
    x[N] = 1.0;
    // interior points: zeros of P_{N-1}^(1,1) (= zeros of P_N'), Newton from
    // the Chebyshev-Gauss-Lobatto points
    for (int i = 1; i < N; ++i) {
        double z = -std::cos(M_PI * i / N);
        for (int it = 0; it < 100; ++it) {
            const double f = jacobi(z, 1, 1, N - 1);
            const double df = jacobi_dx(z, 1, 1, N - 1);
            const double dz = f / df;
            z -= dz;
            if (std::fabs(dz) < 1e-16) break;
        }
        x[i] = z;
    }
    std::sort(x.begin(), x.end());
    return x;
}

// ---------------------------------------------------------------- warp & blend nodes

static const double kAlpha2D[9] = {0, 0.0, 0.0, 1.4152, 0.1001, 0.2751, 0.9800, 1.0999, 1.2832};
static const double kAlpha3D[9] = {0, 0.0, 0.0, 0.0, 0.1002, 1.1332, 1.5608, 1.3413, 1.2577};

// Interpolant (on N+1 equispaced points of [-1,1]) of the shift from those
// points to the LGL points, divided by 1 - x^2; zero at the end points.
struct EdgeWarp {
    int N;
    std::vector<double> xeq, shift;
    explicit EdgeWarp(int n) : N(n), xeq(n + 1), shift(n + 1) {
        std::vector<double> g = lgl_points(n);
        for (int i = 0; i <= n; ++i) {
            xeq[i] = -1.0 + 2.0 * i / n;
            shift[i] = g[i] - xeq[i];
        }
    }
    double operator()(double x) const {
        if (std::fabs(x) >= 1.0 - 1e-10) return 0.0;
        double w = 0.0;
        for (int i = 0; i <= N; ++i) {
            double l = 1.0;
            for (int j = 0; j <= N; ++j)
                if (j != i) l *= (x - xeq[j]) / (xeq[i] - xeq[j]);
            w += shift[i] * l;
        }
        return w / (1.0 - x * x);
    }
};

using Vec3 = std::array<double, 3>;

// Warp of one simplex face (triangle with vertices P[a], P[b], P[c] of side 2):
// each edge (u, v) with opposite face vertex o adds
// 4 lu lv warp(lv - lu) (1 + (alpha lo)^2) along the unit vector u -> v.
static Vec3 face_warp(const EdgeWarp &w, double alpha, const double *lam, const Vec3 *P, int a, int b, int c) {
    const int edge[3][3] = {{a, b, c}, {b, c, a}, {c, a, b}};
    Vec3 d{0, 0, 0};
    for (const auto &e : edge) {
        const int u = e[0], v = e[1], o = e[2];
        Vec3 dir;
        double len = 0;
        for (int k = 0; k < 3; ++k) {
            dir[k] = P[v][k] - P[u][k];
            len += dir[k] * dir[k];
        }
        len = std::sqrt(len);
        const double amt = 4.0 * lam[u] * lam[v] * w(lam[v] - lam[u]) * (1.0 + (alpha * lam[o]) * (alpha * lam[o]));
        for (int k = 0; k < 3; ++k) d[k] += amt * dir[k] / len;
    }
    return d;
}

// Barycentric coordinates of X in the simplex P[0..dim] (dim+1 unknowns).
static void barycentric(int dim, const Vec3 *P, const Vec3 &X, double *lam) {
    Mat A(dim + 1, dim + 1);
    for (int v = 0; v <= dim; ++v) {
        for (int k = 0; k < dim; ++k) A(k, v) = P[v][k];
        A(dim, v) = 1.0;
    }
    Mat Ai = inverse(A);
    for (int v = 0; v <= dim; ++v) {
        double s = Ai(v, dim);
        for (int k = 0; k < dim; ++k) s += Ai(v, k) * X[k];
        lam[v] = s;
    }
}

static void warp_blend_nodes(RefElement &R) {
    const int N = R.N, dim = R.dim;
    const double alpha = dim == 2 ? kAlpha2D[N] : kAlpha3D[N];
    const EdgeWarp w(N);
    const double s3 = std::sqrt(3.0), s6 = std::sqrt(6.0);
    Vec3 P[4] = {{-1, -1 / s3, -1 / s6}, {1, -1 / s3, -1 / s6}, {0, 2 / s3, -1 / s6}, {0, 0, 3 / s6}};
    if (dim == 2) {
        P[0] = {-1, -1 / s3, 0};
        P[1] = {1, -1 / s3, 0};
        P[2] = {0, 2 / s3, 0};
    }
    const double refv[4][3] = {{-1, -1, -1}, {1, -1, -1}, {-1, 1, -1}, {-1, -1, 1}};
    const int nv = dim + 1;
    R.r.assign(R.Np, 0);
    R.s.assign(R.Np, 0);
    R.t.assign(dim == 3 ? R.Np : 0, 0);
    // faces of the tetrahedron: opposite vertex and the three others
    const int tet_faces[4][4] = {{3, 0, 1, 2}, {2, 0, 1, 3}, {0, 1, 2, 3}, {1, 0, 2, 3}};
    const double tol = 1e-10;
    for (int n = 0; n < R.Np; ++n) {
        double lam[4] = {0, 0, 0, 0};
        for (int v = 0; v < nv; ++v) lam[v] = double(R.lattice[n * nv + v]) / N;
        Vec3 X{0, 0, 0};
        for (int v = 0; v < nv; ++v)
            for (int k = 0; k < 3; ++k) X[k] += lam[v] * P[v][k];
        Vec3 shift{0, 0, 0};
        if (dim == 2) {
            shift = face_warp(w, alpha, lam, P, 0, 1, 2);
        } else {
            for (const auto &f : tet_faces) {
                const int o = f[0], a = f[1], b = f[2], c = f[3];
                const Vec3 fw = face_warp(w, alpha, lam, P, a, b, c);
                const double lo = lam[o];
                double blend = lam[a] * lam[b] * lam[c];
                const double den = (lam[a] + 0.5 * lo) * (lam[b] + 0.5 * lo) * (lam[c] + 0.5 * lo);
                if (den > tol) blend = (1.0 + (alpha * lo) * (alpha * lo)) * blend / den;
                const int inner = (lam[a] > tol) + (lam[b] > tol) + (lam[c] > tol);
                if (lo < tol && inner < 3) {
                    shift = fw;  // node on an edge of this face: the edge warp itself
                } else {
                    for (int k = 0; k < 3; ++k) shift[k] += blend * fw[k];
                }
            }
        }
        for (int k = 0; k < 3; ++k) X[k] += shift[k];
        double mu[4];
        barycentric(dim, P, X, mu);
        double rr = 0, ss = 0, tt = 0;
        for (int v = 0; v < nv; ++v) {
            rr += mu[v] * refv[v][0];
            ss += mu[v] * refv[v][1];
            tt += mu[v] * refv[v][2];
        }
        R.r[n] = rr;
        R.s[n] = ss;
        if (dim == 3) R.t[n] = tt;
    }
}

// ---------------------------------------------------------------- orthonormal simplex bases

static double pw(double x, int p) { return p < 0 ? 0.0 : std::pow(x, p); }

// Values and (r,s) gradient of the 2D orthonormal basis at one point.
static void basis2d(int N, double r, double s, double *v, double *vr, double *vs) {
    const double a = std::fabs(1.0 - s) > 1e-14 ? 2.0 * (1.0 + r) / (1.0 - s) - 1.0 : -1.0;
    const double b = s;
    const double c = std::sqrt(2.0);
    int m = 0;
    for (int i = 0; i <= N; ++i)
        for (int j = 0; j <= N - i; ++j, ++m) {
            const double A = jacobi(a, 0, 0, i), dA = jacobi_dx(a, 0, 0, i);
            const double B = jacobi(b, 2 * i + 1, 0, j), dB = jacobi_dx(b, 2 * i + 1, 0, j);
            const double ta = dA * B * pw(1 - b, i - 1);               // (d psi/da)/(1-b) / c
            const double tb = A * (dB * pw(1 - b, i) - i * B * pw(1 - b, i - 1));
            v[m] = c * A * B * pw(1 - b, i);
            vr[m] = c * 2.0 * ta;
            vs[m] = c * ((1 + a) * ta + tb);
        }
}

// Values and (r,s,t) gradient of the 3D orthonormal basis at one point.
static void basis3d(int N, double r, double s, double t, double *v, double *vr, double *vs, double *vt) {
    const double a = std::fabs(s + t) > 1e-14 ? 2.0 * (1.0 + r) / (-s - t) - 1.0 : -1.0;
    const double b = std::fabs(1.0 - t) > 1e-14 ? 2.0 * (1.0 + s) / (1.0 - t) - 1.0 : -1.0;
    const double c = t;
    const double k0 = 2.0 * std::sqrt(2.0);
    int m = 0;
    for (int i = 0; i <= N; ++i)
        for (int j = 0; j <= N - i; ++j)
            for (int k = 0; k <= N - i - j; ++k, ++m) {
                const double A = jacobi(a, 0, 0, i), dA = jacobi_dx(a, 0, 0, i);
                const double Pj = jacobi(b, 2 * i + 1, 0, j), dPj = jacobi_dx(b, 2 * i + 1, 0, j);
                const double Pk = jacobi(c, 2 * i + 2 * j + 2, 0, k), dPk = jacobi_dx(c, 2 * i + 2 * j + 2, 0, k);
                const double B = Pj * pw(1 - b, i);
                const double C = Pk * pw(1 - c, i + j);
                const double dB = dPj * pw(1 - b, i) - i * Pj * pw(1 - b, i - 1);
                const double dC = dPk * pw(1 - c, i + j) - (i + j) * Pk * pw(1 - c, i + j - 1);
                const double ta = dA * Pj * pw(1 - b, i - 1) * Pk * pw(1 - c, i + j - 1);
                const double tb = A * dB * Pk * pw(1 - c, i + j - 1);
                v[m] = k0 * A * B * C;
                vr[m] = k0 * 4.0 * ta;
                vs[m] = k0 * (2.0 * (1 + a) * ta + 2.0 * tb);
                vt[m] = k0 * (2.0 * (1 + a) * ta + (1 + b) * tb + A * B * dC);
            }
}

// ---------------------------------------------------------------- the element

RefElement make_ref_element(int dim, int N) {
    if (dim != 2 && dim != 3) throw std::invalid_argument("dim must be 2 or 3");
    if (N < 1 || N > (dim == 2 ? 8 : 6)) throw std::invalid_argument("order out of range");
    RefElement R;
    R.dim = dim;
    R.N = N;
    const int nv = dim + 1;
    if (dim == 2) {
        R.Np = (N + 1) * (N + 2) / 2;
        R.Nfp = N + 1;
        R.Nfaces = 3;
        for (int j = 0; j <= N; ++j)
            for (int i = 0; i <= N - j; ++i) R.lattice.insert(R.lattice.end(), {N - i - j, i, j});
        R.face_verts = {0, 1, 1, 2, 2, 0};
        R.n_orient = 2;
    } else {
        R.Np = (N + 1) * (N + 2) * (N + 3) / 6;
        R.Nfp = (N + 1) * (N + 2) / 2;
        R.Nfaces = 4;
        for (int k = 0; k <= N; ++k)
            for (int j = 0; j <= N - k; ++j)
                for (int i = 0; i <= N - j - k; ++i) R.lattice.insert(R.lattice.end(), {N - i - j - k, i, j, k});
        R.face_verts = {0, 1, 2, 0, 1, 3, 1, 2, 3, 0, 2, 3};
        R.n_orient = 6;
    }
    warp_blend_nodes(R);

    const int Np = R.Np;
    Mat V(Np, Np), Vr(Np, Np), Vs(Np, Np), Vt(Np, Np);
    for (int n = 0; n < Np; ++n) {
        if (dim == 2)
            basis2d(N, R.r[n], R.s[n], &V.a[(size_t)n * Np], &Vr.a[(size_t)n * Np], &Vs.a[(size_t)n * Np]);
        else
            basis3d(N, R.r[n], R.s[n], R.t[n], &V.a[(size_t)n * Np], &Vr.a[(size_t)n * Np], &Vs.a[(size_t)n * Np],
                    &Vt.a[(size_t)n * Np]);
    }
    const Mat Vi = inverse(V);
    R.Dr = matmul(Vr, Vi);
    R.Ds = matmul(Vs, Vi);
    if (dim == 3) R.Dt = matmul(Vt, Vi);
    R.M = matmul(transpose(Vi), Vi);

    // Face nodes: lattice coordinate of the vertex opposite the face is 0.
    // Order along the face: 2D by the weight of the face's second vertex
    // (traversal v_a -> v_b); 3D by (weight of third, weight of second) vertex.
    const int Nf = R.Nfaces, Nfp = R.Nfp, fv = dim;
    R.face_nodes.assign((size_t)Nf * Nfp, -1);
    std::vector<std::array<int, 3>> face_lat((size_t)Nf * Nfp);
    for (int f = 0; f < Nf; ++f) {
        const int *vf = &R.face_verts[f * fv];
        int opp = 0;
        for (int v = 0; v < nv; ++v) {
            bool in = false;
            for (int q = 0; q < fv; ++q) in = in || vf[q] == v;
            if (!in) opp = v;
        }
        std::vector<std::pair<int, int>> key;  // (sort key, node)
        for (int n = 0; n < Np; ++n) {
            const int *L = &R.lattice[n * nv];
            if (L[opp] != 0) continue;
            const int k = dim == 2 ? L[vf[1]] : L[vf[2]] * (N + 1) + L[vf[1]];
            key.push_back({k, n});
        }
        if ((int)key.size() != Nfp) throw std::runtime_error("face node count");
        std::sort(key.begin(), key.end());
        for (int i = 0; i < Nfp; ++i) {
            const int n = key[i].second;
            R.face_nodes[f * Nfp + i] = n;
            const int *L = &R.lattice[n * nv];
            face_lat[f * Nfp + i] = {L[vf[0]], L[vf[1]], dim == 3 ? L[vf[2]] : 0};
        }
    }
    // Orientation permutations (identical for every face: the face-node
    // order depends only on the face-local lattice).  Orientation o lists the
    // partner face's vertices as a permutation of ours; the partner's node
    // with the same vertex weights is found by lattice match.
    {
        std::vector<std::array<int, 3>> perms;
        if (dim == 2)
            perms = {{0, 1, 2}, {1, 0, 2}};
        else
            perms = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
        R.orient_perm.assign((size_t)R.n_orient * Nfp, -1);
        for (int o = 0; o < R.n_orient; ++o)
            for (int i = 0; i < Nfp; ++i) {
                const auto &l = face_lat[i];  // face 0's lattice order is the generic one
                // partner vertex q is our vertex perms[o][q]
                std::array<int, 3> lp = {l[perms[o][0]], l[perms[o][1]], dim == 3 ? l[perms[o][2]] : 0};
                for (int i2 = 0; i2 < Nfp; ++i2)
                    if (face_lat[i2] == lp) R.orient_perm[o * Nfp + i] = i2;
                if (R.orient_perm[o * Nfp + i] < 0) throw std::runtime_error("orientation table");
            }
    }
    // Combined face mass matrix and LIFT.
    Mat E(Np, Nf * Nfp);
    for (int f = 0; f < Nf; ++f) {
        const int *vf = &R.face_verts[f * fv];
        const int nb = dim == 2 ? N + 1 : (N + 1) * (N + 2) / 2;
        Mat Vf(Nfp, nb);
        std::vector<double> tmp(3 * (size_t)nb);
        for (int i = 0; i < Nfp; ++i) {
            const int n = R.face_nodes[f * Nfp + i];
            // actual barycentric coordinates of the node
            double lam[4];
            lam[1] = 0.5 * (1 + R.r[n]);
            lam[2] = 0.5 * (1 + R.s[n]);
            lam[3] = dim == 3 ? 0.5 * (1 + R.t[n]) : 0.0;
            lam[0] = 1.0 - lam[1] - lam[2] - lam[3];
            if (dim == 2) {
                const double xi = -1.0 + 2.0 * lam[vf[1]];
                for (int m = 0; m < nb; ++m) Vf(i, m) = jacobi(xi, 0, 0, m);
            } else {
                const double u = -1.0 + 2.0 * lam[vf[1]], v = -1.0 + 2.0 * lam[vf[2]];
                basis2d(N, u, v, &Vf.a[(size_t)i * nb], tmp.data(), tmp.data() + nb);
            }
        }
        const Mat Mf = inverse(matmul(Vf, transpose(Vf)));
        for (int i = 0; i < Nfp; ++i)
            for (int j = 0; j < Nfp; ++j) E(R.face_nodes[f * Nfp + i], f * Nfp + j) = Mf(i, j);
    }
    R.LIFT = matmul(matmul(V, transpose(V)), E);
    return R;
}

}  // namespace dgw
