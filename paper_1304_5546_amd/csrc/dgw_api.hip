// C ABI of libdgw.so: solver creation (host FP64 set-up, upload), field
// transfer, the LSRK4 step loop of fused stage kernels, FP64 reductions.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/dgw.h"
#include "device.hpp"
#include "host.hpp"
#include "solver.hpp"

namespace dgw {

// Carpenter & Kennedy (1994) five-stage fourth-order 2N-storage coefficients.
const double kRkA[5] = {0.0, -567301805773.0 / 1357537059087.0, -2404267990393.0 / 2016746695238.0,
                        -3550918686646.0 / 2091501179385.0, -1275806237668.0 / 842570457699.0};
const double kRkB[5] = {1432997174477.0 / 9575080441755.0, 5161836677717.0 / 13612068292357.0,
                        1720146321549.0 / 2090206949498.0, 3134564353537.0 / 4481467310338.0,
                        2277821191437.0 / 14882151754819.0};

}  // namespace dgw

namespace {

thread_local std::string g_last_error;

int fail(int code, const std::string &msg) {
    g_last_error = msg;
    return code;
}

using dgw::kRkA;
using dgw::kRkB;

constexpr int kRedBlocks = 512;

}  // namespace

// Reduction scratch of dgw_energy_noalloc: the per-block partial sums of the
// energy kernel.  A file-scope device array, so that the call allocates
// nothing; every device the library runs on holds its own copy until the
// process ends.  In host code its name is only a stand-in: the device
// address of each device's copy is looked up once per device at solver
// set-up (with that device current) and kept in g_scratch_ptr.
constexpr int kNoAllocPartials = 1024;  // doubles
static __device__ __align__(256) double scratch[kNoAllocPartials];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch_ptr[kMaxDevices] = {};

// Device address of this device's scratch copy; the device must be current.
int init_scratch_ptr(int dev) {
    if (dev < 0 || dev >= kMaxDevices) return fail(DGW_EINVAL, "device ordinal out of range for the scratch table");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr[dev]) return DGW_OK;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
        return fail(DGW_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = (double *)p;
    return DGW_OK;
}

double *scratch_ptr(int dev) {
    if (dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    return g_scratch_ptr[dev];
}

}  // namespace

namespace dgw {

int set_error(int code, const std::string &msg) { return fail(code, msg); }

int64_t solver_footprint(int dim, int order, int64_t K, bool material, int prec) {
    const int64_t Np = dim == 2 ? (order + 1) * (order + 2) / 2 : (order + 1) * (order + 2) * (order + 3) / 6;
    const int64_t Nfp = dim == 2 ? order + 1 : (order + 1) * (order + 2) / 2;
    const int64_t Nf = dim + 1, nf = dim == 2 ? 3 : 6;
    const int64_t G = dim == 2 ? (material ? 6 : 4) : 9, FG = dim == 2 ? (material ? 6 : 3) : 4;
    const int64_t Kp = (K + kTile - 1) / kTile * kTile;
    const int64_t wq = prec == DGW_FP64 ? 8 : 4;        // bytes per field value
    // 3D and 2D FP32 (the element-major kernel may run): nodes padded to 4 per field
    const int64_t npp = (dim == 3 || prec == DGW_FP32) ? dgw::npp_pad((int)Np) : Np;
    int64_t b = 3 * nf * npp * Kp * wq;                  // q ping-pong and res
    b += (G + Nf * FG) * Kp * 4 + Nf * Kp * 4;          // factors and face records
    if (prec != DGW_FP32) b += (G + Nf * FG) * Kp * 8;  // FP64 factors
    const int64_t MT = (Np + 15) / 16, KV = (Np + 3) / 4, KL = (Nf * Nfp + 3) / 4;
    if (prec == DGW_FP64)  // FP64 operators, row-major and in fragment order
        b += Np * (dim * Np + Nf * Nfp) * 8 + (2 * MT * KV + MT * KL) * 64 * 8;
    if (prec == DGW_FP32 && dim == 2) {
        const int64_t KE = dgw::npp_pad((int)Np) / 4;
        b += (2 * MT * KV + MT * KL) * 64 * 4;                                  // derivative-first fragments
        b += (((2 * KE + 3) / 4) * KE + ((KE + 3) / 4) * KL) * 64 * 4;          // element-major fragments
    }
    b += Kp * 4 + Kp * 8 + dim * Np * Kp * 8;           // permutation, J, node coordinates
    if (material) b += nf * Kp * 8;                     // energy weights
    b += 4 * Np * (dim * Np + Nf * Nfp) * 4 + Np * Np * 8 + 64 * 1024;  // operators, tables, scratch
    return b;
}

void steps_for(double t_final, double dt_cfl, int64_t *n, double *dt) {
    int64_t k = (int64_t)std::ceil(t_final / dt_cfl - 1e-12);
    if (k < 1) k = 1;
    *n = t_final == 0 ? 0 : k;
    *dt = t_final / k;
}

}  // namespace dgw

#define DGW_HIP(call)                                                                                     \
    do {                                                                                                  \
        hipError_t e_ = (call);                                                                           \
        if (e_ != hipSuccess) return fail(DGW_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)


namespace {

template <typename T>
int dalloc(T **p, size_t n) {
    if (hipMalloc((void **)p, std::max<size_t>(n, 1) * sizeof(T)) != hipSuccess) {
        *p = nullptr;
        return fail(DGW_ENOMEM, "hipMalloc of " + std::to_string(n * sizeof(T)) + " bytes failed");
    }
    return DGW_OK;
}

template <typename T>
int upload(T *dst, const std::vector<T> &src) {
    DGW_HIP(hipMemcpy(dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice));
    return DGW_OK;
}

// Resident work-groups per CU of the persistent kernel of `variant` on this
// solver (0: the variant is not persistent).
int occupancy_of(const dgw_solver *s, int variant, int pairs, bool share) {
    const bool split = s->opts.prec == DGW_SPLIT_BF16 || s->opts.prec == DGW_SPLIT_FP16;
    if (s->dim == 3) return split ? dgw::blocks_per_cu_3d_split(s->N, share) : dgw::blocks_per_cu_3d(s->N, share);
    if (split) return dgw::blocks_per_cu_2d_split(s->N, s->material, s->opts.prec);
    if (variant == dgw::kVariantScalarOperand) return 0;
    if (variant == dgw::kVariantElemMajor) return dgw::blocks_per_cu_2d_em(s->N, s->material);
    if (s->fp64 || variant == dgw::kVariantDerivFirst)
        return dgw::blocks_per_cu_2d_df(s->N, s->material, s->fp64, s->fp64 ? 1 : pairs);
    return dgw::blocks_per_cu_2d_mfma(s->N, s->material);
}

// Persistent grid of `gpc` work-groups per CU: a multiple of the 8 XCDs, no
// more groups than tiles (rounded up to the 8 XCDs).
void set_grid(dgw_solver *s, int gpc) {
    s->gpc = gpc;
    const int ntiles = (int)(s->Kp / dgw::kTile);
    // work units of the persistent grid: tiles, or windows of several tiles
    const int tpu = s->dim == 2 && s->variant == dgw::kVariantElemMajor ? dgw::tiles_per_group_2d_em(s->N) : 1;
    const int nunits = (ntiles + tpu - 1) / tpu;
    int ng = std::max(1, s->ncu) * std::max(1, gpc);
    ng = std::min(ng, (nunits + 7) / 8 * 8);
    s->ngroups = std::max(8, ng / 8 * 8);
}

void free_device(dgw_solver *s) {
    if (!s->on_device) return;
    hipSetDevice(s->opts.device);
    void *ptrs[] = {s->q[0], s->q[1], s->res, s->geo_d, s->fgeo_d, s->ops_d, s->opsfrag_d, s->nbr_d, s->itab_d, s->perm_d,
                    s->J_d, s->M_d, s->w_d, s->x_d, s->y_d, s->z_d, s->partial_d,
                    s->geo64_d, s->fgeo64_d, s->q64[0], s->q64[1], s->res64, s->ops64_d, s->opsfrag64_d,
                    s->opsfrag_df_d, s->opsfrag_em_d};
    for (void *p : ptrs)
        if (p) hipFree(p);
    if (s->ev0) hipEventDestroy(s->ev0);
    if (s->ev1) hipEventDestroy(s->ev1);
    if (s->own_stream && s->stream) hipStreamDestroy(s->stream);
    s->on_device = false;
}

int setup_device(dgw_solver *s) {
    const int dim = s->dim, Np = s->Np, Nfp = s->Nfp, Nf = s->Nfaces, nf = s->nf;
    const int64_t K = s->K, Kp = s->Kp;
    const auto &g = s->g;
    const auto &R = s->ref;
    DGW_HIP(hipSetDevice(s->opts.device));
    s->on_device = true;
    if (int rc0 = init_scratch_ptr(s->opts.device)) return rc0;
    if (s->opts.hip_stream) {
        s->stream = (hipStream_t)s->opts.hip_stream;
    } else {
        DGW_HIP(hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking));
        s->own_stream = true;
    }
    DGW_HIP(hipEventCreate(&s->ev0));
    DGW_HIP(hipEventCreate(&s->ev1));
    const size_t nstate = s->state_alloc();
    int rc;
    if (s->fp64) {
        if ((rc = dalloc(&s->q64[0], nstate)) || (rc = dalloc(&s->q64[1], nstate)) || (rc = dalloc(&s->res64, nstate)))
            return rc;
        DGW_HIP(hipMemset(s->q64[0], 0, nstate * sizeof(double)));
        DGW_HIP(hipMemset(s->q64[1], 0, nstate * sizeof(double)));
        DGW_HIP(hipMemset(s->res64, 0, nstate * sizeof(double)));
    } else {
        if ((rc = dalloc(&s->q[0], nstate)) || (rc = dalloc(&s->q[1], nstate)) || (rc = dalloc(&s->res, nstate)))
            return rc;
        DGW_HIP(hipMemset(s->q[0], 0, nstate * sizeof(float)));
        DGW_HIP(hipMemset(s->q[1], 0, nstate * sizeof(float)));
        DGW_HIP(hipMemset(s->res, 0, nstate * sizeof(float)));
    }

    // per-element factors
    std::vector<double> geo((size_t)s->G * Kp, 0.0);
    std::vector<double> fgeo((size_t)Nf * s->FG * Kp, 0.0);
    std::vector<int> nbr((size_t)Nf * Kp, -1);
    std::vector<double> J(Kp, 0.0), w(s->material ? (size_t)nf * Kp : 0, 0.0);
    std::vector<double> X((size_t)Np * Kp, 0.0), Y((size_t)Np * Kp, 0.0), Z(dim == 3 ? (size_t)Np * Kp : 0, 0.0);
    const double alpha = s->opts.alpha;
    for (int64_t e = 0; e < K; ++e) {
        const int64_t k = s->perm[e];
        const double *D = &g.drst[(size_t)k * dim * dim];
        for (int c = 0; c < dim * dim; ++c) geo[dgw::tix(e, c, s->G)] = D[c];
        if (dim == 2 && s->material) {
            geo[dgw::tix(e, 4, s->G)] = 1.0 / g.eps[k];
            geo[dgw::tix(e, 5, s->G)] = 1.0 / g.mu[k];
        }
        J[e] = g.J[k];
        if (s->material) {
            // magnetic fields (Hx, Hy[, Hz]) weigh with mu, electric ones with eps
            const int n_h = dim == 2 ? 2 : 3;
            for (int f = 0; f < nf; ++f) w[dgw::tix(e, f, nf)] = (f < n_h) ? g.mu[k] : g.eps[k];
        }
        for (int n = 0; n < Np; ++n) {
            X[dgw::tix(e, n, Np)] = g.x[(size_t)k * Np + n];
            Y[dgw::tix(e, n, Np)] = g.y[(size_t)k * Np + n];
            if (dim == 3) Z[dgw::tix(e, n, Np)] = g.z[(size_t)k * Np + n];
        }
        for (int f = 0; f < Nf; ++f) {
            const size_t kf = (size_t)k * Nf + f;
            const double *nrm = &g.normal[kf * dim];
            const double Fs = g.sJ[kf] / g.J[k];
            // rows face*FG + q of this element are 64 apart in the tiled layout
            double *fg = &fgeo[dgw::tix(e, f * s->FG, Nf * s->FG)];
            for (int c = 0; c < dim; ++c) fg[(size_t)c * 64] = nrm[c];
            const int64_t k2 = g.nbr_elem[kf];
            if (dim == 2 && s->material) {
                // exact upwind (Riemann) flux across the face, blended by
                // alpha with the central flux; Fscale/eps- and Fscale/mu- folded in
                const double Zm = std::sqrt(g.mu[k] / g.eps[k]);
                const double Zp = k2 >= 0 ? std::sqrt(g.mu[k2] / g.eps[k2]) : Zm;
                const double sZ = Zm + Zp;
                const double cEE = alpha / sZ, cEh = 0.5 * (1 - alpha) + alpha * Zp / sZ;
                const double cHE = 0.5 * (1 - alpha) + alpha * Zm / sZ, cHh = alpha * Zm * Zp / sZ;
                fg[(size_t)2 * 64] = Fs / g.eps[k] * cEE;
                fg[(size_t)3 * 64] = Fs / g.eps[k] * cEh;
                fg[(size_t)4 * 64] = Fs / g.mu[k] * cHE;
                fg[(size_t)5 * 64] = Fs / g.mu[k] * cHh;
            } else {
                fg[(size_t)dim * 64] = Fs;
            }
            if (k2 >= 0) {
                const int64_t e2 = s->iperm[k2];
                nbr[dgw::tix(e, f, Nf)] = int((e2 << 5) | (g.nbr_face[kf] << 3) | g.nbr_orient[kf]);
            }
        }
    }
    // operators and tables
    std::vector<float> ops;
    std::vector<double> ops64;
    auto put = [&](const dgw::Mat &M) {
        for (double v : M.a) ops.push_back((float)v);
        ops64.insert(ops64.end(), M.a.begin(), M.a.end());
    };
    put(R.Dr);
    put(R.Ds);
    if (dim == 3) put(R.Dt);
    put(R.LIFT);
    std::vector<int> itab(R.face_nodes.begin(), R.face_nodes.end());
    for (int f2 = 0; f2 < Nf; ++f2)
        for (int o = 0; o < R.n_orient; ++o)
            for (int i = 0; i < Nfp; ++i) itab.push_back(R.face_nodes[f2 * Nfp + R.orient_perm[o * Nfp + i]]);
    std::vector<int> permv(s->perm.begin(), s->perm.end());
    const bool split = s->opts.prec == DGW_SPLIT_BF16 || s->opts.prec == DGW_SPLIT_FP16;
    const bool need64 = s->opts.prec != DGW_FP32;  // FP64 factors on the device
    std::vector<float> opsfrag, opsfrag_df, opsfrag_em;
    std::vector<double> opsfrag64;
    if (s->fp64) {
        // FP64 fragments of the matrix-core kernel (the scalar-operand kernel
        // reads the row-major FP64 operators)
        opsfrag64.resize(dgw::opsfrag2d_df64(s->N, nullptr, nullptr, nullptr, nullptr));
        dgw::opsfrag2d_df64(s->N, R.Dr.a.data(), R.Ds.a.data(), R.LIFT.a.data(), opsfrag64.data());
    } else if (split && dim == 3) {
        const int bytes = dgw::opsfrag3d_split(s->N, nullptr, nullptr, nullptr, nullptr, nullptr);
        opsfrag.resize(bytes / sizeof(float));
        dgw::opsfrag3d_split(s->N, R.Dr.a.data(), R.Ds.a.data(), R.Dt.a.data(), R.LIFT.a.data(), opsfrag.data());
    } else if (split) {
        const int bytes = dgw::opsfrag2d_split(s->N, s->opts.prec, nullptr, nullptr, nullptr, nullptr);
        opsfrag.resize(bytes / sizeof(float));
        dgw::opsfrag2d_split(s->N, s->opts.prec, R.Dr.a.data(), R.Ds.a.data(), R.LIFT.a.data(), opsfrag.data());
        for (int f = 0; f < Nf; ++f)
            for (int i = 0; i < Nfp; ++i)
                if (dgw::face_node2d(s->N, f, i) != R.face_nodes[f * Nfp + i])
                    return fail(DGW_EINVAL, "internal: face node order mismatch");
    } else if (dim == 2) {
        // the MFMA kernel indexes face nodes in closed form: confirm it matches
        for (int f = 0; f < Nf; ++f)
            for (int i = 0; i < Nfp; ++i)
                if (dgw::face_node2d(s->N, f, i) != R.face_nodes[f * Nfp + i])
                    return fail(DGW_EINVAL, "internal: face node order mismatch");
        opsfrag.resize(dgw::opsfrag2d(s->N, nullptr, nullptr, nullptr, nullptr));
        dgw::opsfrag2d(s->N, R.Dr.a.data(), R.Ds.a.data(), R.LIFT.a.data(), opsfrag.data());
        // and those of the derivative-first and element-major kernels, so that
        // any of them can run
        opsfrag_df.resize(dgw::opsfrag2d_df(s->N, nullptr, nullptr, nullptr, nullptr));
        dgw::opsfrag2d_df(s->N, R.Dr.a.data(), R.Ds.a.data(), R.LIFT.a.data(), opsfrag_df.data());
        opsfrag_em.resize(dgw::opsfrag2d_em(s->N, nullptr, nullptr, nullptr, nullptr));
        dgw::opsfrag2d_em(s->N, R.Dr.a.data(), R.Ds.a.data(), R.LIFT.a.data(), opsfrag_em.data());
    } else {
        opsfrag.resize(dgw::opsfrag3d(s->N, nullptr, nullptr, nullptr, nullptr, nullptr));
        dgw::opsfrag3d(s->N, R.Dr.a.data(), R.Ds.a.data(), R.Dt.a.data(), R.LIFT.a.data(), opsfrag.data());
    }

    if ((rc = dalloc(&s->geo_d, geo.size())) || (rc = dalloc(&s->fgeo_d, fgeo.size())) ||
        (rc = dalloc(&s->nbr_d, nbr.size())) || (rc = dalloc(&s->ops_d, ops.size())) ||
        (rc = dalloc(&s->itab_d, itab.size())) || (rc = dalloc(&s->perm_d, permv.size())) ||
        (rc = dalloc(&s->J_d, J.size())) || (rc = dalloc(&s->M_d, R.M.a.size())) ||
        (rc = dalloc(&s->x_d, X.size())) || (rc = dalloc(&s->y_d, Y.size())) ||
        (rc = dalloc(&s->partial_d, 2 * kRedBlocks)) || (rc = dalloc(&s->opsfrag_d, opsfrag.size())))
        return rc;
    if (!opsfrag.empty() && (rc = upload(s->opsfrag_d, opsfrag))) return rc;
    if (!opsfrag_df.empty() &&
        ((rc = dalloc(&s->opsfrag_df_d, opsfrag_df.size())) || (rc = upload(s->opsfrag_df_d, opsfrag_df))))
        return rc;
    if (!opsfrag_em.empty() &&
        ((rc = dalloc(&s->opsfrag_em_d, opsfrag_em.size())) || (rc = upload(s->opsfrag_em_d, opsfrag_em))))
        return rc;
    // persistent grid: every CU filled to its occupancy
    DGW_HIP(hipDeviceGetAttribute(&s->ncu, hipDeviceAttributeMultiprocessorCount, s->opts.device));
    set_grid(s, occupancy_of(s, s->variant, s->pairs, s->share));
    if (dim == 3 && (rc = dalloc(&s->z_d, Z.size()))) return rc;
    if (s->material && (rc = dalloc(&s->w_d, w.size()))) return rc;
    std::vector<float> geo32(geo.begin(), geo.end()), fgeo32(fgeo.begin(), fgeo.end());
    if (need64 && ((rc = dalloc(&s->geo64_d, geo.size())) || (rc = dalloc(&s->fgeo64_d, fgeo.size())) ||
                   (rc = upload(s->geo64_d, geo)) || (rc = upload(s->fgeo64_d, fgeo))))
        return rc;
    if (s->fp64 && ((rc = dalloc(&s->ops64_d, ops64.size())) || (rc = upload(s->ops64_d, ops64)) ||
                    (rc = dalloc(&s->opsfrag64_d, opsfrag64.size())) || (rc = upload(s->opsfrag64_d, opsfrag64))))
        return rc;
    if ((rc = upload(s->geo_d, geo32)) || (rc = upload(s->fgeo_d, fgeo32)) || (rc = upload(s->nbr_d, nbr)) ||
        (rc = upload(s->ops_d, ops)) || (rc = upload(s->itab_d, itab)) || (rc = upload(s->perm_d, permv)) ||
        (rc = upload(s->J_d, J)) || (rc = upload(s->M_d, R.M.a)) || (rc = upload(s->x_d, X)) ||
        (rc = upload(s->y_d, Y)))
        return rc;
    if (dim == 3 && (rc = upload(s->z_d, Z))) return rc;
    if (s->material && (rc = upload(s->w_d, w))) return rc;
    return DGW_OK;
}

int need_device(const dgw_solver *s) {
    if (!s) return fail(DGW_EINVAL, "NULL solver");
    if (!s->on_device) return fail(DGW_ENODEVICE, "solver was created host-only (device = -1)");
    return DGW_OK;
}

dgw::StageArgs stage_args(const dgw_solver *s) {
    dgw::StageArgs a{};
    a.res = s->res;
    a.geo = s->geo_d;
    a.fgeo = s->fgeo_d;
    a.geo64 = s->geo64_d;
    a.fgeo64 = s->fgeo64_d;
    a.nbr = s->nbr_d;
    a.ops = s->ops_d;
    a.opsfrag = s->dim == 2 && !s->fp64 && s->variant == dgw::kVariantDerivFirst ? s->opsfrag_df_d
                : s->dim == 2 && s->variant == dgw::kVariantElemMajor                ? s->opsfrag_em_d
                                                                                     : s->opsfrag_d;
    a.itab = s->itab_d;
    a.Kp = (int)s->Kp;
    a.ntiles = (int)(s->Kp / dgw::kTile);
    a.ngroups = s->ngroups;
    a.alpha = (float)s->opts.alpha;
    a.res64 = s->res64;
    a.ops64 = s->ops64_d;
    a.opsfrag64 = s->opsfrag64_d;
    a.alpha64 = s->opts.alpha;
    return a;
}

// stage input / output buffers and RK coefficients of one launch
void set_stage(const dgw_solver *s, dgw::StageArgs &a, double ca, double cb, double dt) {
    a.qin = s->q[s->cur];
    a.qout = s->q[1 - s->cur];
    a.qin64 = s->q64[s->cur];
    a.qout64 = s->q64[1 - s->cur];
    a.a = (float)ca;
    a.b = (float)cb;
    a.dt = (float)dt;
    a.a64 = ca;
    a.b64 = cb;
    a.dt64 = dt;
}

hipError_t launch_one(const dgw_solver *s, const dgw::StageArgs &a, hipStream_t st) {
    if (s->fp64)
        return s->variant == dgw::kVariantScalarOperand ? dgw::launch_stage2d_fp64(s->N, s->material, a, st)
                                                        : dgw::launch_stage2d_df(s->N, s->material, true, 1, a, st);
    if (s->opts.prec != DGW_FP32)
        return s->dim == 2 ? dgw::launch_stage2d_split(s->N, s->material, s->opts.prec, a, st)
                           : dgw::launch_stage3d_split(s->N, s->share, a, st);
    if (s->dim == 2 && s->variant == dgw::kVariantDerivFirst)
        return dgw::launch_stage2d_df(s->N, s->material, false, s->pairs, a, st);
    if (s->dim == 3) return dgw::launch_stage3d(s->N, s->share, a, st);
    if (s->dim == 2 && s->variant == dgw::kVariantElemMajor) return dgw::launch_stage2d_em(s->N, s->material, a, st);
    return dgw::launch_stage(s->dim, s->N, s->material, s->variant, a, st);
}

int launch_steps_impl(dgw_solver *s, int64_t nsteps, double dt, hipStream_t st) {
    dgw::StageArgs a = stage_args(s);
    for (int64_t n = 0; n < nsteps; ++n)
        for (int st5 = 0; st5 < 5; ++st5) {
            set_stage(s, a, kRkA[st5], kRkB[st5], dt);
            DGW_HIP(launch_one(s, a, st));
            s->cur = 1 - s->cur;
        }
    return DGW_OK;
}

// caller-order FP64 [nf][K][Np] -> internal node-major upload (in the
// solver's field type T) into dst
template <typename T>
int upload_fields_t(dgw_solver *s, const double *q, T *dst) {
    const int Np = s->Np, nf = s->nf;
    const int64_t K = s->K, Kp = s->Kp;
    std::vector<T> h(s->state_size(), T(0));
    for (int f = 0; f < nf; ++f)
        for (int64_t e = 0; e < K; ++e) {
            const int64_t k = s->perm[e];
            const double *src = q + ((size_t)f * K + k) * Np;
            for (int n = 0; n < Np; ++n) h[dgw::fidx(e, f, n, nf, Np, s->npp)] = (T)src[n];
        }
    DGW_HIP(hipMemcpy(dst, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice));
    return DGW_OK;
}

int upload_fields(dgw_solver *s, const double *q) {
    return s->fp64 ? upload_fields_t(s, q, s->q64[s->cur]) : upload_fields_t(s, q, s->q[s->cur]);
}

// zero the RK residual (asynchronously on st)
int clear_res(dgw_solver *s, hipStream_t st) {
    const size_t n = s->state_size();
    if (s->fp64)
        DGW_HIP(hipMemsetAsync(s->res64, 0, n * sizeof(double), st));
    else
        DGW_HIP(hipMemsetAsync(s->res, 0, n * sizeof(float), st));
    return DGW_OK;
}

template <typename T>
int download(dgw_solver *s, const T *src_d, double *out) {
    const int Np = s->Np, nf = s->nf;
    const int64_t K = s->K, Kp = s->Kp;
    std::vector<T> h(s->state_size());
    DGW_HIP(hipStreamSynchronize(s->stream));
    DGW_HIP(hipMemcpy(h.data(), src_d, h.size() * sizeof(T), hipMemcpyDeviceToHost));
    for (int f = 0; f < nf; ++f)
        for (int64_t e = 0; e < K; ++e) {
            const int64_t k = s->perm[e];
            double *dst = out + ((size_t)f * K + k) * Np;
            for (int n = 0; n < Np; ++n) dst[n] = h[dgw::fidx(e, f, n, nf, Np, s->npp)];
        }
    return DGW_OK;
}

double flops_per_element(int dim, int Np, int Nafp, int nf) {
    if (dim == 2) {
        // the paper's model (volume r,s derivatives of 3 fields, chain rule,
        // lift incl. Jacobian, jumps + flux) plus 4 flops per DOF for the RK update
        return 6.0 * 2 * Np * Np + 2.0 * Np * 13 + 3.0 * (2.0 * Np * Nafp + Np) + Nafp * 18.0 + 4.0 * nf * Np;
    }
    // 3D analogue: r,s,t derivatives of 6 fields, chain rule + curl (9 partials
    // per field pair), lift of 6 fluxes, jumps + flux, RK update
    return 18.0 * 2 * Np * Np + 2.0 * Np * 6 * 9 + 6.0 * (2.0 * Np * Nafp + Np) + Nafp * 60.0 + 4.0 * nf * Np;
}

}  // namespace

extern "C" {

const char *dgw_strerror(int code) {
    switch (code) {
        case DGW_OK: return "ok";
        case DGW_EINVAL: return "invalid argument";
        case DGW_EMESH: return "invalid mesh";
        case DGW_EORDER: return "unsupported order";
        case DGW_ENOMEM: return "out of memory";
        case DGW_ETOOBIG: return "footprint too large";
        case DGW_EDEVICE: return "device (HIP) error";
        case DGW_ENONFINITE: return "non-finite field";
        case DGW_ECANCELLED: return "cancelled";
        case DGW_ENOTFOUND: return "not found";
        case DGW_ENODEVICE: return "no device for this handle";
        default: return "unknown error";
    }
}

const char *dgw_last_error(void) { return g_last_error.c_str(); }

int dgw_opts_default(dgw_opts *o) {
    if (!o) return fail(DGW_EINVAL, "NULL opts");
    std::memset(o, 0, sizeof(*o));
    o->alpha = 1.0;
    o->cfl = 1.0;
    o->prec = DGW_FP32;
    o->renumber = 1;
    o->device = 0;
    return DGW_OK;
}

int dgw_reference_element(int32_t dim, int32_t order, int32_t *Np, int32_t *Nfp, double *r, double *s, double *t,
                          double *Dr, double *Ds, double *Dt, double *M, double *LIFT, int32_t *face_nodes) {
    try {
        const dgw::RefElement R = dgw::make_ref_element(dim, order);
        if (Np) *Np = R.Np;
        if (Nfp) *Nfp = R.Nfp;
        auto cp = [](double *d, const std::vector<double> &v) {
            if (d) std::copy(v.begin(), v.end(), d);
        };
        cp(r, R.r);
        cp(s, R.s);
        if (dim == 3) cp(t, R.t);
        cp(Dr, R.Dr.a);
        cp(Ds, R.Ds.a);
        if (dim == 3) cp(Dt, R.Dt.a);
        cp(M, R.M.a);
        cp(LIFT, R.LIFT.a);
        if (face_nodes) std::copy(R.face_nodes.begin(), R.face_nodes.end(), face_nodes);
        return DGW_OK;
    } catch (const std::invalid_argument &e) {
        return fail(dim == 2 || dim == 3 ? DGW_EORDER : DGW_EINVAL, e.what());
    } catch (const std::exception &e) {
        return fail(DGW_EINVAL, e.what());
    }
}

int dgw_create(const dgw_mesh *mesh, int32_t order, const dgw_opts *opts_in, dgw_solver **out) {
    if (!out) return fail(DGW_EINVAL, "NULL output handle");
    *out = nullptr;
    if (!mesh) return fail(DGW_EINVAL, "NULL mesh");
    if (mesh->dim != 2 && mesh->dim != 3) return fail(DGW_EINVAL, "dim must be 2 or 3");
    if (mesh->n_elems <= 0 || mesh->n_verts <= 0) return fail(DGW_EINVAL, "empty mesh");
    if (!mesh->vx || !mesh->vy || (mesh->dim == 3 && !mesh->vz) || !mesh->elem_verts)
        return fail(DGW_EINVAL, "NULL mesh array");
    if (order < 1 || order > (mesh->dim == 2 ? 8 : 4))
        return fail(DGW_EORDER, "order must be in 1..8 (2D) or 1..4 (3D)");
    if (mesh->n_elems >= (int64_t(1) << 26)) return fail(DGW_ETOOBIG, "more than 2^26 elements");
    if (mesh->dim == 2 && !dgw::fits_index32_2d(order, mesh->n_elems))
        return fail(DGW_ETOOBIG, "2D field arrays are limited to 2^32 values (32-bit partner-trace indices)");
    dgw_opts opts;
    dgw_opts_default(&opts);
    if (opts_in) opts = *opts_in;
    if (opts.cfl <= 0) opts.cfl = 1.0;
    if (!(opts.alpha >= 0.0 && opts.alpha <= 1.0)) return fail(DGW_EINVAL, "alpha must be in [0, 1]");
    if (opts.prec != DGW_FP32 && opts.prec != DGW_SPLIT_BF16 && opts.prec != DGW_SPLIT_FP16 && opts.prec != DGW_FP64)
        return fail(DGW_EINVAL, "unknown precision variant");
    if ((opts.prec == DGW_SPLIT_FP16 || opts.prec == DGW_FP64) && mesh->dim != 2)
        return fail(DGW_EINVAL, "the 3D path has the FP32 and split-BF16 variants");
    if (opts.kernel < 0 || opts.kernel > 4) return fail(DGW_EINVAL, "kernel variant must be 0 .. 4");
    if (opts.kernel == 4 && (mesh->dim != 2 || opts.prec != DGW_FP32))
        return fail(DGW_EINVAL, "kernel 4 is the 2D FP32 element-major kernel");
    if ((opts.prec == DGW_SPLIT_BF16 || opts.prec == DGW_SPLIT_FP16) && (opts.kernel == 1 || opts.kernel == 3))
        return fail(DGW_EINVAL, "split-precision variants run on their own matrix-core kernels (kernel 0 or 2)");
    if (opts.kernel == 3 && mesh->dim != 2) return fail(DGW_EINVAL, "kernel 3 is a 2D kernel");
    if (opts.lane_elems < 0 || opts.lane_elems > 2) return fail(DGW_EINVAL, "lane_elems must be 0, 1 or 2");
    if (opts.lane_elems == 2 && (mesh->dim != 2 || opts.prec != DGW_FP32 || (opts.kernel != 0 && opts.kernel != 3)))
        return fail(DGW_EINVAL, "two elements per lane: the 2D derivative-first FP32 kernel only");
    if (opts.wave_private != 0 && opts.wave_private != 1) return fail(DGW_EINVAL, "wave_private must be 0 or 1");
    auto t0 = std::chrono::steady_clock::now();
    dgw_solver *s = new (std::nothrow) dgw_solver();
    if (!s) return fail(DGW_ENOMEM, "host allocation failed");
    s->opts = opts;
    s->fp64 = opts.prec == DGW_FP64;
    // the kernel that runs: 2D FP32 auto = derivative-first up to order 6,
    // fused-operand MFMA above; FP64 auto = derivative-first; split and 3D
    // have one kernel each
    const bool plain32 = opts.prec == DGW_FP32 && mesh->dim == 2;
    s->variant = opts.kernel == dgw::kVariantAuto
                     ? (s->fp64 || (plain32 && dgw::auto_deriv_first(order)) ? dgw::kVariantDerivFirst
                                                                             : dgw::kVariantMfma)
                     : (s->fp64 && opts.kernel == dgw::kVariantMfma ? dgw::kVariantDerivFirst : opts.kernel);
    if (opts.lane_elems == 2) s->variant = dgw::kVariantDerivFirst;
    s->pairs = opts.lane_elems == 2 ? 2 : 1;
    s->share = opts.wave_private == 0;
    s->dim = mesh->dim;
    s->N = order;
    try {
        s->ref = dgw::make_ref_element(mesh->dim, order);
        s->g = dgw::build_geometry(s->ref, mesh->dim, mesh->n_verts, mesh->vx, mesh->vy, mesh->vz, mesh->n_elems,
                                   mesh->elem_verts, mesh->eps, mesh->mu);
    } catch (const dgw::MeshError &e) {
        delete s;
        return fail(e.code == -1 ? DGW_EINVAL : DGW_EMESH, e.msg);
    } catch (const std::bad_alloc &) {
        delete s;
        return fail(DGW_ENOMEM, "host allocation failed during set-up");
    } catch (const std::exception &e) {
        delete s;
        return fail(DGW_EINVAL, e.what());
    }
    s->Np = s->ref.Np;
    s->Nfp = s->ref.Nfp;
    s->Nfaces = s->ref.Nfaces;
    s->nf = s->dim == 2 ? 3 : 6;
    s->K = mesh->n_elems;
    s->Kp = (s->K + dgw::kTile - 1) / dgw::kTile * dgw::kTile;
    s->npp = (s->dim == 3 || s->variant == dgw::kVariantElemMajor) ? dgw::npp_pad(s->Np) : 0;
    if (s->dim == 2 && !s->fp64 && (int64_t)s->state_alloc() * 4 >= (int64_t(1) << 31)) {
        // the element-major kernel addresses partners by 32-bit byte offsets
        if (s->variant == dgw::kVariantElemMajor) {
            delete s;
            return fail(DGW_ETOOBIG, "the element-major 2D kernel is limited to 2 GiB field arrays");
        }
        s->em_ok = false;
    }
    if (s->dim == 3 && (int64_t)s->state_size() * 4 >= (int64_t(1) << 31)) {
        delete s;
        return fail(DGW_ETOOBIG, "3D field arrays are limited to 2 GiB (partner traces use 32-bit byte offsets)");
    }
    for (int64_t k = 0; k < s->K; ++k)
        if (s->g.eps[k] != 1.0 || s->g.mu[k] != 1.0) s->material = true;
    if (s->dim == 3 && s->material) {
        delete s;
        return fail(DGW_EINVAL, "the 3D path supports eps = mu = 1 only");
    }
    s->G = s->dim == 2 ? (s->material ? 6 : 4) : 9;
    s->FG = s->dim == 2 ? (s->material ? 6 : 3) : 4;
    std::vector<int64_t> order_v;
    if (opts.renumber)
        order_v = dgw::morton_order(s->g);
    else {
        order_v.resize(s->K);
        for (int64_t k = 0; k < s->K; ++k) order_v[k] = k;
    }
    s->perm.assign(order_v.begin(), order_v.end());
    s->iperm.assign(s->K, 0);
    for (int64_t e = 0; e < s->K; ++e) s->iperm[s->perm[e]] = (int)e;
    s->dt_cfl = dgw::cfl_dt(s->ref, s->g, opts.cfl);
    if (opts.device >= 0) {
        int rc = setup_device(s);
        if (rc != DGW_OK) {
            free_device(s);
            delete s;
            return rc;
        }
    }
    s->info.setup_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    *out = s;
    return DGW_OK;
}

void dgw_destroy(dgw_solver *s) {
    if (!s) return;
    free_device(s);
    delete s;
}

int dgw_sizes(const dgw_solver *s, int64_t *K, int32_t *Np, int32_t *n_fields) {
    if (!s) return fail(DGW_EINVAL, "NULL solver");
    if (K) *K = s->K;
    if (Np) *Np = s->Np;
    if (n_fields) *n_fields = s->nf;
    return DGW_OK;
}

int dgw_node_coords(const dgw_solver *s, double *x, double *y, double *z) {
    if (!s) return fail(DGW_EINVAL, "NULL solver");
    if (x) std::copy(s->g.x.begin(), s->g.x.end(), x);
    if (y) std::copy(s->g.y.begin(), s->g.y.end(), y);
    if (z && s->dim == 3) std::copy(s->g.z.begin(), s->g.z.end(), z);
    return DGW_OK;
}

int dgw_cfl_dt(const dgw_solver *s, double *dt) {
    if (!s || !dt) return fail(DGW_EINVAL, "NULL argument");
    *dt = s->dt_cfl;
    return DGW_OK;
}

int dgw_set_fields(dgw_solver *s, const double *q) {
    int rc = need_device(s);
    if (rc) return rc;
    if (!q) return fail(DGW_EINVAL, "NULL fields");
    DGW_HIP(hipSetDevice(s->opts.device));
    DGW_HIP(hipStreamSynchronize(s->stream));
    if ((rc = upload_fields(s, q)) || (rc = clear_res(s, s->stream))) return rc;
    DGW_HIP(hipStreamSynchronize(s->stream));
    s->t = 0.0;
    return DGW_OK;
}

int dgw_get_fields(dgw_solver *s, double *q) {
    int rc = need_device(s);
    if (rc) return rc;
    if (!q) return fail(DGW_EINVAL, "NULL fields");
    DGW_HIP(hipSetDevice(s->opts.device));
    return s->fp64 ? download(s, s->q64[s->cur], q) : download(s, s->q[s->cur], q);
}

int dgw_set_cavity_mode(dgw_solver *s, const int32_t mode[3]) {
    int rc = need_device(s);
    if (rc) return rc;
    if (!mode) return fail(DGW_EINVAL, "NULL mode");
    DGW_HIP(hipSetDevice(s->opts.device));
    dgw::CavityArgs a{};
    a.npp = s->npp;
    a.q = s->q[s->cur];
    a.q64 = s->q64[s->cur];
    a.x = s->x_d;
    a.y = s->y_d;
    a.z = s->z_d;
    a.Kp = (int)s->Kp;
    a.K = (int)s->K;
    a.Np = s->Np;
    a.dim = s->dim;
    a.m = mode[0];
    a.n = mode[1];
    a.l = s->dim == 3 ? mode[2] : 0;
    a.eps = s->g.eps[0];
    a.mu = s->g.mu[0];
    a.t = 0.0;
    DGW_HIP(dgw::launch_cavity_init(a, s->stream));
    if ((rc = clear_res(s, s->stream))) return rc;
    DGW_HIP(hipStreamSynchronize(s->stream));
    s->t = 0.0;
    return DGW_OK;
}

int dgw_advance_steps(dgw_solver *s, int64_t nsteps, double dt) {
    int rc = need_device(s);
    if (rc) return rc;
    if (nsteps < 0) return fail(DGW_EINVAL, "negative step count");
    if (dt <= 0) dt = s->dt_cfl;
    DGW_HIP(hipSetDevice(s->opts.device));
    DGW_HIP(hipEventRecord(s->ev0, s->stream));
    if ((rc = launch_steps_impl(s, nsteps, dt, s->stream))) return rc;
    DGW_HIP(hipEventRecord(s->ev1, s->stream));
    DGW_HIP(hipEventSynchronize(s->ev1));
    float ms = 0.0f;
    DGW_HIP(hipEventElapsedTime(&ms, s->ev0, s->ev1));
    s->t += nsteps * dt;
    s->info.steps = nsteps;
    s->info.dt = dt;
    s->info.t = s->t;
    s->info.solve_ms = ms;
    s->info.dof_updates_per_s = ms > 0 ? double(s->nf) * s->K * s->Np * nsteps / (ms * 1e-3) : 0.0;
    return DGW_OK;
}

int dgw_advance(dgw_solver *s, double t_final, double dt, int64_t *steps_taken) {
    int rc = need_device(s);
    if (rc) return rc;
    if (!(t_final >= 0)) return fail(DGW_EINVAL, "t_final must be >= 0");
    int64_t n;
    if (dt <= 0) {
        dgw::steps_for(t_final, s->dt_cfl, &n, &dt);
    } else {
        n = (int64_t)std::llround(t_final / dt);
        if (t_final == 0) n = 0;
    }
    if ((rc = dgw_advance_steps(s, n, dt))) return rc;
    if (steps_taken) *steps_taken = n;
    return DGW_OK;
}

int dgw_rhs(dgw_solver *s, const double *q, double *rhs) {
    int rc = need_device(s);
    if (rc) return rc;
    if (!q || !rhs) return fail(DGW_EINVAL, "NULL argument");
    if ((rc = dgw_set_fields(s, q))) return rc;
    dgw::StageArgs a = stage_args(s);
    set_stage(s, a, 0.0, 0.0, 1.0);
    DGW_HIP(launch_one(s, a, s->stream));
    s->cur = 1 - s->cur;
    return s->fp64 ? download(s, s->res64, rhs) : download(s, s->res, rhs);
}

int dgw_energy(dgw_solver *s, double *energy) {
    int rc = need_device(s);
    if (rc) return rc;
    if (!energy) return fail(DGW_EINVAL, "NULL output");
    DGW_HIP(hipSetDevice(s->opts.device));
    dgw::ReduceArgs a{};
    a.npp = s->npp;
    a.q = s->q[s->cur];
    a.q64 = s->q64[s->cur];
    a.J = s->J_d;
    a.Mref = s->M_d;
    a.w = s->w_d;
    a.Kp = (int)s->Kp;
    a.K = (int)s->K;
    a.Np = s->Np;
    a.nf = s->nf;
    a.partial = s->partial_d;
    DGW_HIP(dgw::launch_energy(a, kRedBlocks, s->stream));
    std::vector<double> h(kRedBlocks);
    DGW_HIP(hipStreamSynchronize(s->stream));
    DGW_HIP(hipMemcpy(h.data(), s->partial_d, kRedBlocks * sizeof(double), hipMemcpyDeviceToHost));
    double e = 0.0;
    for (double v : h) e += v;
    *energy = 0.5 * e;
    if (!std::isfinite(*energy)) return fail(DGW_ENONFINITE, "energy is not finite");
    return DGW_OK;
}

int dgw_energy_noalloc(dgw_solver *s, double *energy_dev, void *stream) {
    int rc = need_device(s);
    if (rc) return rc;
    if (!energy_dev) return fail(DGW_EINVAL, "NULL output");
    static_assert(kRedBlocks <= kNoAllocPartials, "energy partials exceed the static scratch");
    if (kRedBlocks > kNoAllocPartials)
        return fail(DGW_ETOOBIG, "energy reduction needs more partials than the static scratch holds");
    double *ptr = scratch_ptr(s->opts.device);
    if (!ptr) return fail(DGW_EDEVICE, "scratch address of this device not set up");
    DGW_HIP(hipSetDevice(s->opts.device));
    hipStream_t st = stream ? (hipStream_t)stream : s->stream;
    dgw::ReduceArgs a{};
    a.npp = s->npp;
    a.q = s->q[s->cur];
    a.q64 = s->q64[s->cur];
    a.J = s->J_d;
    a.Mref = s->M_d;
    a.w = s->w_d;
    a.Kp = (int)s->Kp;
    a.K = (int)s->K;
    a.Np = s->Np;
    a.nf = s->nf;
    a.partial = ptr;  // every block writes its slot: nothing to clear
    DGW_HIP(dgw::launch_energy(a, kRedBlocks, st));
    DGW_HIP(dgw::launch_sum_partials(ptr, kRedBlocks, 0.5, energy_dev, st));
    return DGW_OK;
}

int dgw_cavity_error(dgw_solver *s, const int32_t mode[3], double t, double *rel_l2) {
    int rc = need_device(s);
    if (rc) return rc;
    if (!mode || !rel_l2) return fail(DGW_EINVAL, "NULL argument");
    DGW_HIP(hipSetDevice(s->opts.device));
    dgw::CavityArgs a{};
    a.npp = s->npp;
    a.q = s->q[s->cur];
    a.q64 = s->q64[s->cur];
    a.x = s->x_d;
    a.y = s->y_d;
    a.z = s->z_d;
    a.J = s->J_d;
    a.Mref = s->M_d;
    a.Kp = (int)s->Kp;
    a.K = (int)s->K;
    a.Np = s->Np;
    a.dim = s->dim;
    a.m = mode[0];
    a.n = mode[1];
    a.l = s->dim == 3 ? mode[2] : 0;
    a.eps = s->g.eps[0];
    a.mu = s->g.mu[0];
    a.t = t;
    a.partial = s->partial_d;
    DGW_HIP(dgw::launch_cavity_error(a, kRedBlocks, s->stream));
    std::vector<double> h(2 * kRedBlocks);
    DGW_HIP(hipStreamSynchronize(s->stream));
    DGW_HIP(hipMemcpy(h.data(), s->partial_d, h.size() * sizeof(double), hipMemcpyDeviceToHost));
    double num = 0.0, den = 0.0;
    for (int b = 0; b < kRedBlocks; ++b) {
        num += h[2 * b];
        den += h[2 * b + 1];
    }
    *rel_l2 = den > 0 ? std::sqrt(num / den) : std::sqrt(num);
    if (!std::isfinite(*rel_l2)) return fail(DGW_ENONFINITE, "error is not finite");
    return DGW_OK;
}

int dgw_last_info(const dgw_solver *s, dgw_info *info) {
    if (!s || !info) return fail(DGW_EINVAL, "NULL argument");
    *info = s->info;
    info->kernel = s->variant;
    info->groups_per_cu = s->gpc;
    info->lane_elems = s->pairs;
    info->wave_private = s->share ? 0 : 1;
    return DGW_OK;
}

int dgw_set_fields_dev(dgw_solver *s, const float *q_dev, void *stream) {
    int rc = need_device(s);
    if (rc) return rc;
    if (!q_dev) return fail(DGW_EINVAL, "NULL fields");
    if (s->fp64) return fail(DGW_EINVAL, "FP32 device fields given to an FP64 solver");
    hipStream_t st = stream ? (hipStream_t)stream : s->stream;
    DGW_HIP(hipSetDevice(s->opts.device));
    DGW_HIP(dgw::launch_to_internal(q_dev, s->q[s->cur], s->perm_d, (int)s->K, (int)s->Kp, s->Np, s->nf,
                                    s->npp, st));
    if ((rc = clear_res(s, st))) return rc;
    s->t = 0.0;
    return DGW_OK;
}

int dgw_get_fields_dev(dgw_solver *s, float *q_dev, void *stream) {
    int rc = need_device(s);
    if (rc) return rc;
    if (!q_dev) return fail(DGW_EINVAL, "NULL fields");
    if (s->fp64) return fail(DGW_EINVAL, "FP32 device fields requested from an FP64 solver");
    hipStream_t st = stream ? (hipStream_t)stream : s->stream;
    DGW_HIP(hipSetDevice(s->opts.device));
    DGW_HIP(dgw::launch_to_caller(s->q[s->cur], q_dev, s->perm_d, (int)s->K, (int)s->Kp, s->Np, s->nf,
                                    s->npp, st));
    return DGW_OK;
}

int dgw_launch_steps(dgw_solver *s, int64_t nsteps, double dt, void *stream) {
    int rc = need_device(s);
    if (rc) return rc;
    if (nsteps < 0 || !(dt > 0)) return fail(DGW_EINVAL, "nsteps >= 0 and dt > 0 required");
    DGW_HIP(hipSetDevice(s->opts.device));
    hipStream_t st = stream ? (hipStream_t)stream : s->stream;
    if ((rc = launch_steps_impl(s, nsteps, dt, st))) return rc;
    s->t += nsteps * dt;
    return DGW_OK;
}

int dgw_autotune(dgw_solver *s, int32_t stages, dgw_tune_info *out) {
    int rc = need_device(s);
    if (rc) return rc;
    if (stages <= 0) stages = 10;
    DGW_HIP(hipSetDevice(s->opts.device));
    DGW_HIP(hipStreamSynchronize(s->stream));
    // the candidates: every stage kernel of this dimension and arithmetic
    // with its work partitions (elements per lane, shared or wave-private
    // windows), each persistent one at every work-group count per CU up to
    // its occupancy
    struct Cand {
        int variant, gpc, pairs;
        bool share;
    };
    std::vector<Cand> cand;
    struct Part {
        int variant, pairs;
        bool share;
    };
    std::vector<Part> parts;
    const bool split = s->opts.prec == DGW_SPLIT_BF16 || s->opts.prec == DGW_SPLIT_FP16;
    if (s->dim == 3) {
        parts = {{s->variant, 1, true}, {s->variant, 1, false}};
    } else if (split) {
        parts = {{s->variant, 1, true}};
    } else if (s->fp64) {
        parts = {{dgw::kVariantDerivFirst, 1, true}, {dgw::kVariantScalarOperand, 1, true}};
    } else {
        parts = {{dgw::kVariantMfma, 1, true}, {dgw::kVariantDerivFirst, 1, true}, {dgw::kVariantDerivFirst, 2, true},
                 {dgw::kVariantScalarOperand, 1, true}};
        if (s->em_ok) parts.push_back({dgw::kVariantElemMajor, 1, true});
    }
    for (const Part &p : parts) {
        const int occ = occupancy_of(s, p.variant, p.pairs, p.share);
        if (occ == 0)
            cand.push_back({p.variant, 0, p.pairs, p.share});
        else
            for (int g = 1; g <= std::min(occ, 4); ++g) cand.push_back({p.variant, g, p.pairs, p.share});
    }
    if ((int)cand.size() > DGW_TUNE_MAX) cand.resize(DGW_TUNE_MAX);
    // save the state (fields, residual, ping-pong index), try every
    // candidate on the solver's own buffers, restore the state bitwise
    const size_t nstate = s->state_size(), bytes = nstate * (s->fp64 ? 8 : 4);
    void *cur_d = s->fp64 ? (void *)s->q64[s->cur] : (void *)s->q[s->cur];
    void *res_d = s->fp64 ? (void *)s->res64 : (void *)s->res;
    void *save = nullptr;
    if (hipMalloc(&save, 2 * bytes) != hipSuccess) return fail(DGW_ENOMEM, "autotune: no device memory for the saved state");
    struct Free {
        void *p;
        ~Free() { hipFree(p); }
    } free_save{save};
    const int cur0 = s->cur, var0 = s->variant, gpc0 = s->gpc, npp0 = s->npp, pairs0 = s->pairs;
    const bool share0 = s->share;
    DGW_HIP(hipMemcpyAsync(save, cur_d, bytes, hipMemcpyDeviceToDevice, s->stream));
    DGW_HIP(hipMemcpyAsync((char *)save + bytes, res_d, bytes, hipMemcpyDeviceToDevice, s->stream));
    dgw_tune_info info{};
    int best = -1;
    double best_us = 0;
    const double dt = s->dt_cfl;
    // a failing step ends the search; the state is restored either way
    auto try_hip = [&](hipError_t e, const char *what) {
        if (e != hipSuccess && !rc) rc = fail(DGW_EDEVICE, std::string("autotune: ") + what + ": " + hipGetErrorString(e));
        return rc == DGW_OK;
    };
    // candidates run on the solver's buffers whatever their layout (the
    // values only need to be finite for timing; the saved state is restored
    // in the chosen kernel's layout at the end)
    for (size_t i = 0; i < cand.size() && rc == DGW_OK; ++i) {
        s->variant = cand[i].variant;
        s->pairs = cand[i].pairs;
        s->share = cand[i].share;
        set_grid(s, cand[i].gpc);
        dgw::StageArgs a = stage_args(s);
        auto run = [&](int n) {
            for (int k = 0; k < n && rc == DGW_OK; ++k) {
                set_stage(s, a, kRkA[k % 5], kRkB[k % 5], dt);
                try_hip(launch_one(s, a, s->stream), "stage launch");
                s->cur = 1 - s->cur;
            }
            return rc == DGW_OK;
        };
        float ms = 0;
        if (!run(2) || !try_hip(hipEventRecord(s->ev0, s->stream), "event") || !run(stages) ||
            !try_hip(hipEventRecord(s->ev1, s->stream), "event") ||
            !try_hip(hipEventSynchronize(s->ev1), "event synchronisation") ||
            !try_hip(hipEventElapsedTime(&ms, s->ev0, s->ev1), "event timing"))
            break;
        const double us = 1e3 * ms / stages;
        info.tried_kernel[i] = cand[i].variant;
        info.tried_groups_per_cu[i] = cand[i].gpc;
        info.tried_lane_elems[i] = cand[i].pairs;
        info.tried_wave_private[i] = cand[i].share ? 0 : 1;
        info.tried_us[i] = us;
        info.n_tried = (int)i + 1;
        if (best < 0 || us < best_us) {
            best = (int)i;
            best_us = us;
        }
    }
    // keep the fastest candidate (or the old choice on error) and restore the
    // state in its field layout
    const bool ok = rc == DGW_OK && best >= 0;
    s->variant = ok ? cand[best].variant : var0;
    s->pairs = ok ? cand[best].pairs : pairs0;
    s->share = ok ? cand[best].share : share0;
    s->npp = (s->dim == 3 || s->variant == dgw::kVariantElemMajor) ? dgw::npp_pad(s->Np) : 0;
    set_grid(s, ok ? cand[best].gpc : gpc0);
    s->cur = cur0;
    cur_d = s->fp64 ? (void *)s->q64[s->cur] : (void *)s->q[s->cur];
    if (s->npp == npp0) {
        try_hip(hipMemcpyAsync(cur_d, save, bytes, hipMemcpyDeviceToDevice, s->stream), "state restore");
        try_hip(hipMemcpyAsync(res_d, (char *)save + bytes, bytes, hipMemcpyDeviceToDevice, s->stream), "state restore");
    } else {
        const float *sv = static_cast<const float *>(save);
        try_hip(dgw::launch_relayout(sv, (float *)cur_d, (int)s->Kp, s->Np, s->nf, npp0, s->npp, s->stream),
                "state restore");
        try_hip(dgw::launch_relayout(sv + nstate, (float *)res_d, (int)s->Kp, s->Np, s->nf, npp0, s->npp, s->stream),
                "state restore");
    }
    try_hip(hipStreamSynchronize(s->stream), "synchronisation");
    if (!ok) return rc ? rc : fail(DGW_EINVAL, "autotune: no candidate");
    info.kernel = s->variant;
    info.groups_per_cu = s->gpc;
    info.lane_elems = s->pairs;
    info.wave_private = s->share ? 0 : 1;
    info.best_us = best_us;
    if (out) *out = info;
    return DGW_OK;
}

int dgw_stage_cost(const dgw_solver *s, double *bytes, double *flops) {
    if (!s) return fail(DGW_EINVAL, "NULL solver");
    const int Nafp = s->Nfaces * s->Nfp;
    // algorithmic HBM traffic per element: read q_in and res, write res and
    // q_out (4 words per DOF, FP32 or FP64) plus the per-element and per-face
    // factors (FP32, or FP64 in the split-precision and FP64 variants) and
    // the face records
    const double wg = s->opts.prec == DGW_FP32 ? 4.0 : 8.0;
    const double wq = s->fp64 ? 8.0 : 4.0;
    const double per_el = 4.0 * wq * s->nf * s->Np + wg * s->G + s->Nfaces * (wg * s->FG + 4.0);
    if (bytes) *bytes = per_el * double(s->K);
    if (flops) *flops = flops_per_element(s->dim, s->Np, Nafp, s->nf) * double(s->K);
    return DGW_OK;
}

}  // extern "C"
