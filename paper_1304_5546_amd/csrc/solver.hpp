// Library-internal state of one solve (the opaque dgw_solver of the C ABI),
// shared by the solver calls and the request server.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/dgw.h"
#include "device.hpp"
#include "host.hpp"

struct dgw_solver {
    dgw::RefElement ref;
    dgw::Geometry g;
    int dim = 2, N = 1, Np = 0, Nfp = 0, Nfaces = 0, nf = 0;
    int64_t K = 0, Kp = 0;
    int npp = 0;  // field layout (dgw::fidx): 0 = 2D tiled; 3D and the 2D element-major
                  // kernel: padded nodes per field
    // values in one field array (q, res) in the current layout
    size_t state_size() const { return npp ? (size_t)Kp * nf * npp : (size_t)nf * Np * Kp; }
    // values allocated per field array: enough for either layout of a 2D FP32
    // solve (the kernel, and with it the layout, may change by autotuning)
    size_t state_alloc() const { return fp64 ? state_size() : (size_t)Kp * nf * ((Np + 3) / 4 * 4); }
    int G = 0, FG = 0;
    bool material = false;
    dgw_opts opts{};
    std::vector<int> perm;   // internal e -> caller k
    std::vector<int> iperm;  // caller k -> internal e
    double dt_cfl = 0.0;
    int ngroups = 8;  // persistent grid size
    bool on_device = false;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    bool fp64 = false;  // DGW_FP64: fields in q64 / res64, FP32 q / res unused
    int variant = 2;   // 2D stage kernel that runs (dgw::StageVariant, resolved)
    bool em_ok = true; // the element-major 2D kernel may run (field arrays below 2 GiB)
    int pairs = 1;     // elements per lane of the 2D derivative-first FP32 kernel (1 or 2)
    bool share = true; // 3D: the work-group's pair of tiles shared through LDS
    int ncu = 0, gpc = 0;  // CUs of the device, persistent work-groups per CU
    float *q[2] = {nullptr, nullptr};
    float *res = nullptr;
    double *q64[2] = {nullptr, nullptr};
    double *res64 = nullptr, *ops64_d = nullptr, *opsfrag64_d = nullptr;
    float *opsfrag_df_d = nullptr;  // FP32 2D: fragments of the derivative-first kernel
    float *opsfrag_em_d = nullptr;  // FP32 2D: fragments of the element-major kernel
    int cur = 0;
    float *geo_d = nullptr, *fgeo_d = nullptr, *ops_d = nullptr, *opsfrag_d = nullptr;
    double *geo64_d = nullptr, *fgeo64_d = nullptr;  // split-precision and FP64 variants only
    int *nbr_d = nullptr, *itab_d = nullptr, *perm_d = nullptr;
    double *J_d = nullptr, *M_d = nullptr, *w_d = nullptr, *x_d = nullptr, *y_d = nullptr, *z_d = nullptr;
    double *partial_d = nullptr;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    dgw_info info{};
    double t = 0.0;
};

namespace dgw {

// Carpenter & Kennedy (1994) five-stage fourth-order 2N-storage coefficients.
extern const double kRkA[5];
extern const double kRkB[5];

// Device bytes a solver of this size allocates (fields, factors, tables,
// coordinates, reduction scratch).
int64_t solver_footprint(int dim, int order, int64_t K, bool material, int prec);

// Set the calling thread's last-error text; returns code.
int set_error(int code, const std::string &msg);

// Step count and step for reaching t_final at (at most) the CFL step.
void steps_for(double t_final, double dt_cfl, int64_t *n, double *dt);

}  // namespace dgw
