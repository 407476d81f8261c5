// Device-side data layout and launch wrappers of the fused LSRK stage.
//
// HBM layout (internal element order e = 0..Kp-1, Kp = K rounded up to the
// 64-element tile; padding elements carry zero fields and geometry).  Every
// per-element array is tiled, [tile][row][64] (see tix()), so that one wave's
// 64 lanes (64 consecutive elements of a tile) read one row as 256
// contiguous bytes:
//   q, res  : rows f*Np + n, FP32 (n_fields*Np rows; FP64 in FP64 solvers)
//   geo     : G rows of per-element factors: 2D r_x, r_y, s_x, s_y (+ 1/eps,
//             1/mu with materials); 3D the nine entries of A_k^{-1}
//   fgeo    : Nfaces*FG rows of per-face data, row face*FG + q: 2D n_x, n_y,
//             Fscale, or n_x, n_y and four flux coefficients with materials;
//             3D n_x, n_y, n_z, Fscale
//   nbr     : Nfaces rows of int32 face records: -1 on the PEC wall, else
//             (e' << 5) | (f' << 3) | orientation
//   ops     : FP32 Dr, Ds (, Dt) [Np][Np] and LIFT [Np][Nfaces*Nfp], row-major
//   itab    : int32 own face nodes [Nfaces*Nfp], then the partner node table
//             [Nfaces][n_orient][Nfp] (volume node of the partner's face node)
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace dgw {

constexpr int kTile = 64;  // elements per work-group tile (one per lane)

// Tiled (AoSoA) index of row `row` of element e in an array with `rows` rows
// per element: [tile][row][64 elements].  One row of a tile is 256 contiguous
// bytes (a coalesced wave access) and all rows of a tile form one contiguous
// chunk, so a tile touches few pages whatever the mesh size.
__host__ __device__ inline size_t tix(int64_t e, int row, int rows) {
    return ((size_t)(e >> 6) * rows + row) * 64 + (size_t)(e & 63);
}

// Field arrays (q, res).  2D: the tiled layout, row f*Np + n of element e
// at tix(e, f*Np + n, nf*Np).  3D: element-major, element e's fields one
// after another, each padded to npp = Np rounded up to 4 nodes
// ([e][f][npp], the pad nodes hold 0): one element's values form one
// contiguous block, so the face traces of a partner element touch a few
// cache lines instead of one line per node.  npp == 0 selects the 2D form.
__host__ __device__ inline size_t fidx(int64_t e, int f, int n, int nf, int Np, int npp) {
    return npp ? ((size_t)e * nf + f) * npp + n : tix(e, f * Np + n, nf * Np);
}
__host__ __device__ constexpr int npp_pad(int Np) { return (Np + 3) / 4 * 4; }

// Nodes owned by lane group g (g = 0..3, lanes 16 g .. 16 g + 15) in the 3D
// kernels: slot i = 0..kv-1 (kv = npp / 4) holds node slot_node(kv, g, i).
// Slots come in runs of four consecutive nodes (one 16-byte access per
// lane), 16 nodes per run of the four lane groups; the remaining kv mod 4
// slots hold nodes 16 (kv/4) + 4 r + g.  Over the four lane groups every
// node 0..npp-1 appears once.
__host__ __device__ constexpr int slot_node(int kv, int g, int i) {
    return i < 4 * (kv / 4) ? 16 * (i / 4) + 4 * g + (i % 4) : 16 * (kv / 4) + 4 * (i - 4 * (kv / 4)) + g;
}

// The 2D fused-operand and split kernels address partner traces by 32-bit
// element indices into the [tile][3 Np][64] field array: true when the array
// of a 2D solve of order N on K elements stays below 2^32 values.
inline bool fits_index32_2d(int N, int64_t K) {
    const int64_t Np = (int64_t)(N + 1) * (N + 2) / 2, Kp = (K + 63) / 64 * 64;
    return 3 * Np * Kp < (int64_t(1) << 32);
}

// One solve inside a batched stage launch: its buffers, its first tile in
// the launch's global tile numbering, and its time step.
struct BatchDesc {
    float *q[2];          // ping-pong field buffers
    float *res;
    const float *geo;
    const float *fgeo;
    const int *nbr;
    int tile0;            // first global tile of this solve
    int cur0;             // q[cur0 ^ parity] is the stage input
    float dt;
    float pad_;
};

struct StageArgs {
    const float *qin;
    float *qout;
    float *res;
    const float *geo;
    const float *fgeo;
    const int *nbr;
    const float *ops;
    const float *opsfrag;  // operators in MFMA A-fragment order, laid out for the launched kernel
    const int *itab;
    const double *geo64;   // FP64 copies of geo / fgeo (split-precision kernels)
    const double *fgeo64;
    const BatchDesc *batch;  // batched launches: per-solve descriptors
    const int *tile_req;     // batched launches: solve index of every tile
    int parity;              // batched launches: stage count since cur0, mod 2
    // FP64 field path: fields, residual and operators in FP64 (factors in
    // geo64 / fgeo64), RK coefficients and flux parameter in FP64
    const double *qin64;
    double *qout64;
    double *res64;
    const double *ops64;       // row-major Dr, Ds, LIFT (scalar-operand kernel)
    const double *opsfrag64;   // A-fragment order (derivative-first FP64 kernel)
    double a64, b64, dt64, alpha64;
    int Kp;
    int ntiles;
    int ngroups;  // work-groups of a persistent launch (multiple of 8)
    float a, b, dt, alpha;
};

// Kernel variants of the fused stage (2D): fused-operand producer/consumer
// MFMA kernel, scalar-operand VALU kernel, derivative-first MFMA kernel.
// Variant 4 runs on the element-major field layout (fidx with npp > 0).
enum StageVariant {
    kVariantAuto = 0,
    kVariantScalarOperand = 1,
    kVariantMfma = 2,
    kVariantDerivFirst = 3,
    kVariantElemMajor = 4
};

// Launch one fused stage: res <- a res + dt L(qin); qout <- qin + b res.
hipError_t launch_stage(int dim, int N, bool material, int variant, const StageArgs &args, hipStream_t stream);
const char *stage_kernel_name(int dim, int N, bool material, int variant);

hipError_t launch_stage2d_mfma(int N, bool material, const StageArgs &a, hipStream_t s);
// One stage over several solves of the same order and material class at once
// (a.batch / a.tile_req / a.parity, a.ntiles = total tiles; a.dt unused).
hipError_t launch_stage2d_batch(int N, bool material, const StageArgs &a, hipStream_t s);
int blocks_per_cu_2d_batch(int N, bool material);
// fragment-ordered fused operator [Dr | Ds | LIFT] (see stage2d_mfma.hip);
// with out == nullptr returns the required length
int opsfrag2d(int N, const double *Dr, const double *Ds, const double *LIFT, float *out);
int face_node2d(int N, int f, int t);
// operator fragments of the 3D FP32 kernel (packed [Dr; Ds; Dt], LIFT; see
// stage3d.hip); with out == nullptr returns the number of floats
int opsfrag3d(int N, const double *Dr, const double *Ds, const double *Dt, const double *LIFT, float *out);
// resident work-groups per CU of the persistent 2D MFMA kernel
int blocks_per_cu_2d_mfma(int N, bool material);
// 3D: share = partner traces of the work-group's pair of tiles from the
// other waves' LDS copies (else each wave alone, no work-group barriers)
int blocks_per_cu_3d(int N, bool share);
hipError_t launch_stage3d(int N, bool share, const StageArgs &a, hipStream_t s);

// FP64 2D stage on FP64 fields (a.qin64 / a.qout64 / a.res64, a.geo64 /
// a.fgeo64, a.a64 / a.b64 / a.dt64 / a.alpha64, row-major a.ops64): the
// scalar-operand kernel
hipError_t launch_stage2d_fp64(int N, bool material, const StageArgs &a, hipStream_t s);
// Derivative-first 2D MFMA stage, persistent grid of a.ngroups work-groups:
// FP32 (a.qin / ..., operator fragments a.opsfrag) or FP64 (a.qin64 / ...,
// a.opsfrag64)
// pairs: elements per lane, 1 or (FP32 only) 2
hipError_t launch_stage2d_df(int N, bool material, bool fp64, int pairs, const StageArgs &a, hipStream_t s);
int blocks_per_cu_2d_df(int N, bool material, bool fp64, int pairs);
// the 2D FP32 kernel that runs by default: derivative-first up to order 6,
// fused-operand from order 7 (measured: faster at every order on 131k
// elements, slower at order 7 on 524k)
inline bool auto_deriv_first(int N) { return N <= 6; }
// its fragment-ordered Dr, Ds, LIFT; with out == nullptr returns the length
int opsfrag2d_df(int N, const double *Dr, const double *Ds, const double *LIFT, float *out);
int opsfrag2d_df64(int N, const double *Dr, const double *Ds, const double *LIFT, double *out);

// Element-major 2D FP32 stage (variant 4; fields in the fidx layout with
// npp = npp_pad(Np)), persistent grid whose work-groups walk windows of
// tiles_per_group_2d_em(N) tiles, and its operator fragments (with out ==
// nullptr returns the number of floats)
hipError_t launch_stage2d_em(int N, bool material, const StageArgs &a, hipStream_t s);
int blocks_per_cu_2d_em(int N, bool material);
int tiles_per_group_2d_em(int N);
int opsfrag2d_em(int N, const double *Dr, const double *Ds, const double *LIFT, float *out);
// Copy a field array between the two field layouts (same element order):
// src in the layout of npp_src, dst in that of npp_dst (0: tiled).
hipError_t launch_relayout(const float *src, float *dst, int Kp, int Np, int nf, int npp_src, int npp_dst,
                           hipStream_t stream);

// Split-precision 2D stage (prec 1 = BF16 hi+lo, 2 = FP16 hi+lo), FP32
// accumulation, FP64 geometric factors (geo64 / fgeo64).
hipError_t launch_stage2d_split(int N, bool material, int prec, const StageArgs &a, hipStream_t s);
int blocks_per_cu_2d_split(int N, bool material, int prec);
// 16-bit hi/lo operator fragments of the 2D split kernel (Dr, Ds, LIFT given
// row-major in FP64); with out == nullptr returns the required size in bytes
int opsfrag2d_split(int N, int prec, const double *Dr, const double *Ds, const double *LIFT, void *out);
// Split-BF16 3D stage (FP64 geo64 / fgeo64) and its operator fragments
hipError_t launch_stage3d_split(int N, bool share, const StageArgs &a, hipStream_t s);
int blocks_per_cu_3d_split(int N, bool share);
int opsfrag3d_split(int N, const double *Dr, const double *Ds, const double *Dt, const double *LIFT, void *out);

// FP64 reductions: per-block partial sums of
//   energy: J_k sum_f w_f q_f^T M q_f     (w from wvec: [n_fields][Kp] FP64 or NULL = 1)
// into partial[nblocks].
struct ReduceArgs {
    int npp;              // field layout (fidx): 0 = 2D tiled, else the 3D padded node count
    const float *q;
    const double *q64;    // FP64 fields (FP64 solvers; q unused then)
    const double *J;      // [Kp]
    const double *Mref;   // [Np][Np]
    const double *w;      // [n_fields][Kp] or nullptr
    int Kp, K, Np, nf;
    double *partial;
};
hipError_t launch_energy(const ReduceArgs &a, int nblocks, hipStream_t stream);
// *out = scale * (partial[0] + partial[1] + ... + partial[n-1]), summed in
// index order by one device thread
hipError_t launch_sum_partials(const double *partial, int n, double scale, double *out, hipStream_t stream);

// Relative L2 vs the closed-form cavity mode at time t: partial[2*b] is the
// error mass norm squared, partial[2*b+1] the reference's.
struct CavityArgs {
    int npp;              // field layout (fidx): 0 = 2D tiled, else the 3D padded node count
    float *q;             // fields (written by init, read by error)
    double *q64;          // FP64 fields instead (FP64 solvers)
    const double *x, *y, *z;   // node coordinates [Np][Kp]
    const double *J;
    const double *Mref;
    int Kp, K, Np, dim;
    int m, n, l;
    double eps, mu, t;
    double *partial;
};
hipError_t launch_cavity_init(const CavityArgs &a, hipStream_t stream);
hipError_t launch_cavity_error(const CavityArgs &a, int nblocks, hipStream_t stream);

// Layout permutation between the caller's [nf][K][Np] FP32 and the internal
// field layout (fidx with npp); perm[e] = caller element at internal e (e < K).
hipError_t launch_to_internal(const float *src, float *dst, const int *perm, int K, int Kp, int Np, int nf, int npp,
                              hipStream_t stream);
hipError_t launch_to_caller(const float *src, float *dst, const int *perm, int K, int Kp, int Np, int nf, int npp,
                            hipStream_t stream);

}  // namespace dgw
