// Host-side (FP64) set-up of the nodal DG discretisation: reference element,
// per-element geometry, face connectivity, element renumbering, CFL step.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace dgw {

// Dense row-major matrix helper.
struct Mat {
    int rows = 0, cols = 0;
    std::vector<double> a;
    Mat() = default;
    Mat(int r, int c) : rows(r), cols(c), a((size_t)r * c, 0.0) {}
    double &operator()(int i, int j) { return a[(size_t)i * cols + j]; }
    double operator()(int i, int j) const { return a[(size_t)i * cols + j]; }
};

Mat matmul(const Mat &A, const Mat &B);
Mat transpose(const Mat &A);
// Inverse by Gauss-Jordan elimination with partial pivoting; throws on a
// singular matrix.
Mat inverse(const Mat &A);

// Nodal reference simplex of order N (dim 2 or 3).
struct RefElement {
    int dim = 2, N = 1, Np = 0, Nfp = 0, Nfaces = 0;
    std::vector<double> r, s, t;          // node coordinates
    std::vector<int> lattice;             // Np x (dim+1) barycentric lattice ints
    Mat Dr, Ds, Dt, M, LIFT;              // LIFT: Np x Nfaces*Nfp
    std::vector<int> face_nodes;          // Nfaces x Nfp volume-node ids
    // face f: local (reference) vertex ids spanning it, dim entries each
    std::vector<int> face_verts;          // Nfaces x dim
    // neighbour face-node permutation: for each orientation id o and face
    // node i, the index on the partner face (see orientation()).
    int n_orient = 0;
    std::vector<int> orient_perm;         // n_orient x Nfp
};

// Throws std::invalid_argument for an unsupported order.
RefElement make_ref_element(int dim, int N);

// Legendre-Gauss-Lobatto points of degree N, ascending (Newton iteration).
std::vector<double> lgl_points(int N);

// Mesh-level set-up (everything in FP64, element order = caller order).
struct Geometry {
    int dim = 2;
    int64_t K = 0;
    std::vector<double> J;                 // K
    std::vector<double> drst;              // K x dim*dim: row-major d(r,s,t)/d(x,y,z)
    std::vector<double> normal;            // K x Nfaces x dim (outward unit)
    std::vector<double> sJ;                // K x Nfaces
    std::vector<double> x, y, z;           // K x Np node coordinates
    std::vector<int64_t> nbr_elem;         // K x Nfaces: partner element or -1 (PEC)
    std::vector<int> nbr_face;             // K x Nfaces
    std::vector<int> nbr_orient;           // K x Nfaces
    std::vector<double> inradius;          // K
    std::vector<double> eps, mu;           // K
};

// Throws std::invalid_argument (message) on a bad mesh; code set in *err.
Geometry build_geometry(const RefElement &ref, int dim, int64_t n_verts, const double *vx,
                        const double *vy, const double *vz, int64_t K, const int32_t *ev,
                        const double *eps, const double *mu);

// Element order along a Morton (Z-order) curve of the vertex centroids:
// returns order[i] = caller element placed at internal position i.
std::vector<int64_t> morton_order(const Geometry &g);

double cfl_dt(const RefElement &ref, const Geometry &g, double cfl_factor);

struct MeshError {
    int code;
    std::string msg;
};

}  // namespace dgw
