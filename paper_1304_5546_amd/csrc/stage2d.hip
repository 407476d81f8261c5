// Fused LSRK stage for 2D TM Maxwell on triangles, gfx950, on FP32 fields
// (a cross-check of the MFMA kernel) or FP64 fields (the double-precision
// path: fields, residual, operators, factors and arithmetic all FP64).
//
// One work-group (4 waves) owns a tile of 64 consecutive elements; lane l of
// every wave works on element tile*64 + l, so every global access to the
// node-major fields is a 256-byte contiguous row.  Per stage it computes the
// semi-discrete right-hand side of eq. dg-strong-explicit and the 2N-storage
// RK update in one pass over HBM:
//   1. stage the tile's fields q_in (3 x Np x 64) in LDS;
//   2. face gather + upwind flux (eq. max2d-numflux with the factor 1/2,
//      [q] = q^- - q^+; PEC mirror state on the wall; exact Riemann flux across
//      eps/mu jumps): wave w takes face nodes w, w+4, ...; own traces come from
//      LDS, the partner's from q_in in HBM/L2 through the compressed face
//      record (partner element, face, orientation) and a small partner-node
//      table; the scaled fluxes go to LDS;
//   3. local differentiation: wave w takes output nodes w, w+4, ... and
//      accumulates Dr q and Ds q for the three fields; the operator entries
//      are wave-uniform, so they are fetched by scalar loads and feed the FMAs
//      as scalar operands; the chain rule (eq. dg-diff-local-to-global)
//      forms -dEz/dy, dEz/dx, dHy/dx - dHx/dy;
//   4. LIFT apply of the LDS fluxes (eq. dg-lift), same operand scheme;
//   5. res <- a res + dt rhs;  q_out <- q_in + b res  (res prefetched in 1.).
#include <hip/hip_runtime.h>

#include "device.hpp"

namespace dgw {

// Blocks are dispatched round-robin over the 8 XCDs of MI355X; give each XCD
// a contiguous range of tiles so that neighbour traces are shared in its L2.
__device__ __forceinline__ int xcd_tile(int b, int nb) {
    const int x = b & 7, i = b >> 3, q = nb >> 3, r = nb & 7;
    return x * q + (x < r ? x : r) + i;
}

// The solve's buffers and coefficients in the arithmetic type R.
template <typename R>
struct Bufs {
    const R *qin;
    R *qout, *res;
    const R *geo, *fgeo, *ops;
    R a, b, dt, alpha;
};

template <typename R>
__host__ __device__ __forceinline__ Bufs<R> bufs(const StageArgs &A) {
    if constexpr (sizeof(R) == 8)
        return Bufs<R>{A.qin64, A.qout64, A.res64, A.geo64, A.fgeo64, A.ops64, A.a64, A.b64, A.dt64, A.alpha64};
    else
        return Bufs<R>{A.qin, A.qout, A.res, A.geo, A.fgeo, A.ops, A.a, A.b, A.dt, A.alpha};
}

template <typename R, int N, bool MAT>
__global__ void __launch_bounds__(256) stage2d_kernel(StageArgs SA) {
    const Bufs<R> A = bufs<R>(SA);
    constexpr int Np = (N + 1) * (N + 2) / 2;
    constexpr int Nfp = N + 1;
    constexpr int Nafp = 3 * Nfp;
    constexpr int NW = 4;
    constexpr int NR = (Np + NW - 1) / NW;  // output nodes per wave
    constexpr int FG = MAT ? 6 : 3;
    constexpr int TE = kTile;

    __shared__ R sq[3 * Np * TE];
    __shared__ R sf[3 * Nafp * TE];
    __shared__ int stab[3 * 2 * Nfp];

    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int e = tile * TE + lane;

    for (int i = threadIdx.x; i < 3 * 2 * Nfp; i += 256) stab[i] = SA.itab[Nafp + i];

    // 1. fields of the tile into LDS; prefetch this wave's residual entries
#pragma unroll
    for (int row = w; row < 3 * Np; row += NW) sq[row * TE + lane] = A.qin[tix(e, row, 3 * Np)];
    R rres[3][NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        const int n = (w + NW * r < Np) ? w + NW * r : Np - 1;
#pragma unroll
        for (int f = 0; f < 3; ++f) rres[f][r] = A.res[tix(e, f * Np + n, 3 * Np)];
    }
    __syncthreads();

    // 2. face gather and flux
#pragma unroll
    for (int j = w; j < Nafp; j += NW) {
        const int face = j / Nfp, i = j - face * Nfp;
        const int own = SA.itab[j];
        const R mHx = sq[(0 * Np + own) * TE + lane];
        const R mHy = sq[(1 * Np + own) * TE + lane];
        const R mEz = sq[(2 * Np + own) * TE + lane];
        const int rec = SA.nbr[tix(e, face, 3)];
        R pHx, pHy, pEz;
        if (rec < 0) {  // PEC wall: mirror state E+ = -E-, H+ = H-
            pHx = mHx;
            pHy = mHy;
            pEz = -mEz;
        } else {
            const int e2 = rec >> 5, f2 = (rec >> 3) & 3, o = rec & 7;
            const int pn = stab[(f2 * 2 + o) * Nfp + i];
            pHx = A.qin[tix(e2, 0 * Np + pn, 3 * Np)];
            pHy = A.qin[tix(e2, 1 * Np + pn, 3 * Np)];
            pEz = A.qin[tix(e2, 2 * Np + pn, 3 * Np)];
        }
        const R *fg = A.fgeo + tix(e, face * FG, 3 * FG);  // rows face*FG + q are 64 apart
        const R nx = fg[0], ny = fg[64];
        const R dHx = mHx - pHx, dHy = mHy - pHy, dEz = mEz - pEz;
        const R dh = nx * dHy - ny * dHx;  // jump of the tangential field
        R cEE, cEh, cHE, cHh;
        if (MAT) {
            cEE = fg[2 * 64];
            cEh = fg[3 * 64];
            cHE = fg[4 * 64];
            cHh = fg[5 * 64];
        } else {
            const R hs = R(0.5) * fg[2 * 64];
            cEE = A.alpha * hs;
            cEh = hs;
            cHE = hs;
            cHh = A.alpha * hs;
        }
        const R fE = -(cEE * dEz + cEh * dh);
        const R fH = cHE * dEz + cHh * dh;
        sf[(0 * Nafp + j) * TE + lane] = ny * fH;
        sf[(1 * Nafp + j) * TE + lane] = -nx * fH;
        sf[(2 * Nafp + j) * TE + lane] = fE;
    }
    __syncthreads();

    // 3. local differentiation of the three fields for this wave's nodes
    const R *Dr = A.ops;
    const R *Ds = A.ops + Np * Np;
    const R *L = A.ops + 2 * Np * Np;
    R ar[3][NR], as[3][NR];
#pragma unroll
    for (int r = 0; r < NR; ++r)
#pragma unroll
        for (int f = 0; f < 3; ++f) ar[f][r] = as[f][r] = R(0);
#pragma unroll
    for (int jn = 0; jn < Np; ++jn) {
        const R v0 = sq[(0 * Np + jn) * TE + lane];
        const R v1 = sq[(1 * Np + jn) * TE + lane];
        const R v2 = sq[(2 * Np + jn) * TE + lane];
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            const int n = (w + NW * r < Np) ? w + NW * r : Np - 1;
            const R cr = Dr[n * Np + jn], cs = Ds[n * Np + jn];
            ar[0][r] += cr * v0;
            as[0][r] += cs * v0;
            ar[1][r] += cr * v1;
            as[1][r] += cs * v1;
            ar[2][r] += cr * v2;
            as[2][r] += cs * v2;
        }
    }
    constexpr int G = MAT ? 6 : 4;
    const R rx = A.geo[tix(e, 0, G)], ry = A.geo[tix(e, 1, G)];
    const R sx = A.geo[tix(e, 2, G)], sy = A.geo[tix(e, 3, G)];
    R rhs[3][NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        rhs[0][r] = -(ry * ar[2][r] + sy * as[2][r]);
        rhs[1][r] = rx * ar[2][r] + sx * as[2][r];
        rhs[2][r] = (rx * ar[1][r] + sx * as[1][r]) - (ry * ar[0][r] + sy * as[0][r]);
    }
    if (MAT) {
        const R ieps = A.geo[tix(e, 4, G)], imu = A.geo[tix(e, 5, G)];
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            rhs[0][r] *= imu;
            rhs[1][r] *= imu;
            rhs[2][r] *= ieps;
        }
    }

    // 4. LIFT apply
#pragma unroll
    for (int j = 0; j < Nafp; ++j) {
        const R f0 = sf[(0 * Nafp + j) * TE + lane];
        const R f1 = sf[(1 * Nafp + j) * TE + lane];
        const R f2 = sf[(2 * Nafp + j) * TE + lane];
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            const int n = (w + NW * r < Np) ? w + NW * r : Np - 1;
            const R c = L[n * Nafp + j];
            rhs[0][r] += c * f0;
            rhs[1][r] += c * f1;
            rhs[2][r] += c * f2;
        }
    }

    // 5. fused low-storage RK update
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        const int n = w + NW * r;
        if (n < Np) {
#pragma unroll
            for (int f = 0; f < 3; ++f) {
                const size_t idx = tix(e, f * Np + n, 3 * Np);
                const R rr = A.a * rres[f][r] + A.dt * rhs[f][r];
                A.res[idx] = rr;
                A.qout[idx] = sq[(f * Np + n) * TE + lane] + A.b * rr;
            }
        }
    }
}

template <typename R, int N, bool MAT>
static hipError_t launch2d(const StageArgs &a, hipStream_t s) {
    const Bufs<R> b = bufs<R>(a);
    if (a.ntiles <= 0 || !b.qin || !b.qout || !b.res || !b.geo || !b.fgeo || !b.ops || !a.nbr || !a.itab)
        return hipErrorInvalidValue;
    hipLaunchKernelGGL((stage2d_kernel<R, N, MAT>), dim3(a.ntiles), dim3(256), 0, s, a);
    return hipGetLastError();
}

const char *stage3d_kernel_name(int N);

hipError_t launch_stage(int dim, int N, bool material, int variant, const StageArgs &a, hipStream_t s) {
    if (dim == 3) return launch_stage3d(N, true, a, s);
    if (variant != kVariantScalarOperand) return launch_stage2d_mfma(N, material, a, s);
#define DGW_CASE(n)                                                    \
    case n:                                                            \
        return material ? launch2d<float, n, true>(a, s) : launch2d<float, n, false>(a, s);
    switch (N) {
        DGW_CASE(1)
        DGW_CASE(2)
        DGW_CASE(3)
        DGW_CASE(4)
        DGW_CASE(5)
        DGW_CASE(6)
        DGW_CASE(7)
        DGW_CASE(8)
        default:
            return hipErrorInvalidValue;
    }
#undef DGW_CASE
}

hipError_t launch_stage2d_fp64(int N, bool material, const StageArgs &a, hipStream_t s) {
#define DGW_CASE(n)                                                    \
    case n:                                                            \
        return material ? launch2d<double, n, true>(a, s) : launch2d<double, n, false>(a, s);
    switch (N) {
        DGW_CASE(1)
        DGW_CASE(2)
        DGW_CASE(3)
        DGW_CASE(4)
        DGW_CASE(5)
        DGW_CASE(6)
        DGW_CASE(7)
        DGW_CASE(8)
        default:
            return hipErrorInvalidValue;
    }
#undef DGW_CASE
}

const char *stage_kernel_name(int dim, int N, bool material, int variant) {
    (void)N;
    if (dim == 3) return stage3d_kernel_name(N);
    if (variant == kVariantElemMajor) return material ? "stage2d_em_kernel<N, true>" : "stage2d_em_kernel<N, false>";
    if (variant != kVariantScalarOperand) return material ? "stage2d_mfma_kernel<N, true, false>" : "stage2d_mfma_kernel<N, false, false>";
    return material ? "stage2d_kernel<float, N, true>" : "stage2d_kernel<float, N, false>";
}

}  // namespace dgw
