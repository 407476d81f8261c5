// Fused LSRK stage for 3D Maxwell on tetrahedra (eps = mu = 1), FP32, with
// the element-local contractions on the matrix cores (v_mfma_f32_16x16x4_f32).
//
// 3D analogue of eq. dg-strong-explicit (section "Adding Generality": the
// kernels change only mildly): with the fused operator Op = [Dr | Ds | Dt |
// LIFT] (Np x (3 Np + 4 Nfp)) and g_p = (p_x, p_y, p_z) the gradient of the
// reference coordinate p in {r, s, t} (constant on an affine element),
//   curl E = sum_p D_p (g_p x E),
// so each output field is one contraction:
//   rhs_H = Op [-(g_r x E); -(g_s x E); -(g_t x E); flux_H]
//   rhs_E = Op [ (g_r x H);  (g_s x H);  (g_t x H); flux_E]
// with the upwind flux (3D form of eq. max2d-numflux, factor 1/2):
//   flux_H = Fscale/2 ( n x [E] + alpha (n (n.[H]) - [H]) )
//   flux_E = Fscale/2 (-n x [H] + alpha (n (n.[E]) - [E]) ).
//
// Work-group = 4 waves, tile = 64 consecutive elements, wave w owns the MFMA
// N-tile of elements 16w..16w+15.  (1) All waves stage the tile's fields and
// the partner traces of every face node in LDS (the partner's node through
// the face record and the orientation table; on the PEC wall the mirror state
// E+ = -E-, H+ = H-).  (2) Each wave evaluates the flux of its 16 elements in
// place of their partner traces.  (3) Contraction over the volume and flux
// columns, the A fragments of Op streamed from L1/L2 several K-steps ahead.
// The kernel is persistent: a work-group walks a contiguous run of tiles of
// its XCD's share of the mesh.
// (4) res <- a res + dt rhs, q_out <- q_in + b res.
#include <hip/hip_runtime.h>

#include "device.hpp"

namespace dgw {

typedef float floatx4 __attribute__((ext_vector_type(4)));

namespace {

template <int N>
struct Tet {
    static constexpr int Np = (N + 1) * (N + 2) * (N + 3) / 6;
    static constexpr int Nfp = (N + 1) * (N + 2) / 2;
    static constexpr int Nafp = 4 * Nfp;
    static constexpr int Kd = 3 * Np + Nafp;
    static constexpr int KS = (Kd + 3) / 4;
    static constexpr int MT = (Np + 15) / 16;
    static constexpr int RP = 6 * Np;        // partner-trace / flux rows start
    static constexpr int R = RP + 6 * Nafp;  // LDS rows of the tile
    static constexpr int SUB = R * 16 + ((R & 1) ? 0 : 16);
    static constexpr int NT = Nafp + 4 * 6 * Nfp;  // face-node tables
};

}  // namespace

template <int N>
__global__ void __launch_bounds__(256) stage3d_kernel(StageArgs A) {
    using T = Tet<N>;
    constexpr int Np = T::Np, Nfp = T::Nfp, Nafp = T::Nafp, Kd = T::Kd, KS = T::KS, MT = T::MT;
    constexpr int RP = T::RP, SUB = T::SUB, NT = T::NT;
    __shared__ float sq[4 * SUB];
    __shared__ int stab[NT];

    const int lane0 = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int g0 = lane0 >> 4, c0 = lane0 & 15;
    const int col0 = 16 * w + c0;

    for (int i = threadIdx.x; i < NT; i += 256) stab[i] = A.itab[i];

    // tiles of this XCD: a contiguous range, dealt round-robin to its groups
    const int x = blockIdx.x & 7, bi = blockIdx.x >> 3, GB = gridDim.x >> 3;
    const int q8 = A.ntiles >> 3, r8 = A.ntiles & 7;
    const int xbase = x * q8 + (x < r8 ? x : r8), xcount = q8 + (x < r8 ? 1 : 0);
    for (int tl = bi; tl < xcount; tl += GB) {
    const int tile = xbase + tl;
    __syncthreads();  // previous tile's readers of the LDS tile are done
    // lane indices opaque to the compiler: per-lane offsets are recomputed per
    // tile instead of being hoisted out of the tile loop into long-lived registers
    int lane = lane0, col = col0, g = g0, c = c0;
    asm volatile("" : "+v"(lane), "+v"(col), "+v"(g), "+v"(c));

    // ---- (1) stage fields and partner traces (lane <-> element `lane`).
    // Loads are issued in compile-time batches so that a whole batch is in
    // flight before the first of its LDS stores waits.
    {
        constexpr int QW = (6 * Np + 3) / 4;  // field rows per wave
        constexpr int QB = 28;                // rows per batch
        constexpr int JW = (Nafp + 3) / 4;    // face nodes per wave
        constexpr int JB = 5;                 // face nodes per batch (x6 fields)
        const float *qt = A.qin + (size_t)tile * (6 * Np * 64);
        float *L = sq + (lane >> 4) * SUB + (lane & 15);
        const int *nt = A.nbr + (size_t)tile * (4 * 64);
        int rec[4];
#pragma unroll
        for (int f = 0; f < 4; ++f) rec[f] = nt[(unsigned)(f * 64 + lane)];
#pragma unroll
        for (int i0 = 0; i0 < QW; i0 += QB) {
            float v[QB];
#pragma unroll
            for (int i = 0; i < QB; ++i) {
                const int r = w + 4 * (i0 + i);
                v[i] = (i0 + i < QW && r < 6 * Np) ? qt[(unsigned)(r * 64 + lane)] : 0.f;
            }
#pragma unroll
            for (int i = 0; i < QB; ++i) {
                const int r = w + 4 * (i0 + i);
                if (i0 + i < QW && r < 6 * Np) L[r * 16] = v[i];
            }
        }
        __syncthreads();  // stab visible
#pragma unroll
        for (int j0 = 0; j0 < JW; j0 += JB) {
            float v[JB][6];
            bool wl[JB];
#pragma unroll
            for (int jj = 0; jj < JB; ++jj) {
                const int j = w + 4 * (j0 + jj);
                wl[jj] = false;
#pragma unroll
                for (int f = 0; f < 6; ++f) v[jj][f] = 0.f;
                if (j0 + jj < JW && j < Nafp) {
                    const int face = j / Nfp, i = j - face * Nfp;
                    const int rc = face == 0 ? rec[0] : face == 1 ? rec[1] : face == 2 ? rec[2] : rec[3];
                    const bool wall = rc < 0;
                    const int e2 = wall ? tile * 64 + lane : (rc >> 5);
                    const int pn = wall ? stab[j] : stab[Nafp + (((rc >> 3) & 3) * 6 + (rc & 7)) * Nfp + i];
                    const unsigned q0 = ((unsigned)(e2 >> 6) * (6 * Np) + pn) * 64 + (e2 & 63);
#pragma unroll
                    for (int f = 0; f < 6; ++f) v[jj][f] = A.qin[q0 + f * Np * 64];
                    wl[jj] = wall;
                }
            }
#pragma unroll
            for (int jj = 0; jj < JB; ++jj) {
                const int j = w + 4 * (j0 + jj);
                if (j0 + jj < JW && j < Nafp) {
#pragma unroll
                    for (int f = 0; f < 6; ++f)  // PEC mirror: E+ = -E-, H+ = H-
                        L[(RP + f * Nafp + j) * 16] = (wl[jj] && f >= 3) ? -v[jj][f] : v[jj][f];
                }
            }
        }
    }

    // per-column data of this wave's 16 elements
    const float *gt = A.geo + (size_t)tile * (9 * 64);
    float G[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) G[q] = gt[(unsigned)(q * 64 + col)];
    const float *ft = A.fgeo + (size_t)tile * (16 * 64);
    float FD[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) FD[q] = ft[(unsigned)(q * 64 + col)];
    __syncthreads();

    float *B = sq + w * SUB + c;  // this wave's sub-tile, column c

    // ---- (2) upwind flux of this wave's elements, in place of the partner traces
    const float ha = 0.5f * A.alpha;
    for (int jb = 0; jb < (Nafp + 3) / 4; ++jb) {
        const int j = 4 * jb + g;
        if (j < Nafp) {
            const int face = j / Nfp;
            const int own = stab[j];
            float m[6], d[6];
#pragma unroll
            for (int f = 0; f < 6; ++f) {
                m[f] = B[(f * Np + own) * 16];
                d[f] = m[f] - B[(RP + f * Nafp + j) * 16];
            }
            const float nx = face == 0 ? FD[0] : face == 1 ? FD[4] : face == 2 ? FD[8] : FD[12];
            const float ny = face == 0 ? FD[1] : face == 1 ? FD[5] : face == 2 ? FD[9] : FD[13];
            const float nz = face == 0 ? FD[2] : face == 1 ? FD[6] : face == 2 ? FD[10] : FD[14];
            const float fs = face == 0 ? FD[3] : face == 1 ? FD[7] : face == 2 ? FD[11] : FD[15];
            const float dHx = d[0], dHy = d[1], dHz = d[2], dEx = d[3], dEy = d[4], dEz = d[5];
            const float ndH = nx * dHx + ny * dHy + nz * dHz;
            const float ndE = nx * dEx + ny * dEy + nz * dEz;
            const float h = 0.5f * fs, ah = ha * fs;
            // n x [E], n x [H]
            const float cEx = ny * dEz - nz * dEy, cEy = nz * dEx - nx * dEz, cEz = nx * dEy - ny * dEx;
            const float cHx = ny * dHz - nz * dHy, cHy = nz * dHx - nx * dHz, cHz = nx * dHy - ny * dHx;
            B[(RP + 0 * Nafp + j) * 16] = h * cEx + ah * (nx * ndH - dHx);
            B[(RP + 1 * Nafp + j) * 16] = h * cEy + ah * (ny * ndH - dHy);
            B[(RP + 2 * Nafp + j) * 16] = h * cEz + ah * (nz * ndH - dHz);
            B[(RP + 3 * Nafp + j) * 16] = -h * cHx + ah * (nx * ndE - dEx);
            B[(RP + 4 * Nafp + j) * 16] = -h * cHy + ah * (ny * ndE - dEy);
            B[(RP + 5 * Nafp + j) * 16] = -h * cHz + ah * (nz * ndE - dEz);
        }
    }
    // the flux rows read below are this wave's own: LDS order within a wave suffices

    // ---- (3) contraction on the matrix cores
    floatx4 acc[6][MT];
#pragma unroll
    for (int f = 0; f < 6; ++f)
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) acc[f][mt] = floatx4{0.f, 0.f, 0.f, 0.f};
    // The A fragments stream from L1/L2 through a PD-deep software pipeline
    // (the LDS holds the tile; the whole operator does not fit in registers
    // next to the 6 x MT accumulators).
    constexpr int PD = 6;
    float apipe[PD][MT];
#pragma unroll
    for (int d = 0; d < PD; ++d)
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) apipe[d][mt] = d < KS ? A.opsfrag[(unsigned)((mt * KS + d) * 64 + lane)] : 0.f;
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
        float a[MT];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
            a[mt] = apipe[ks % PD][mt];
            if (ks + PD < KS) apipe[ks % PD][mt] = A.opsfrag[(unsigned)((mt * KS + ks + PD) * 64 + lane)];
        }
        const int k = 4 * ks + g;
        float b[6];
        if (k < 3 * Np) {
            const int p = k / Np, node = k - p * Np;
            const float gx = p == 0 ? G[0] : p == 1 ? G[3] : G[6];
            const float gy = p == 0 ? G[1] : p == 1 ? G[4] : G[7];
            const float gz = p == 0 ? G[2] : p == 1 ? G[5] : G[8];
            float v[6];
#pragma unroll
            for (int f = 0; f < 6; ++f) v[f] = B[(f * Np + node) * 16];
            // -(g x E) for the H outputs, (g x H) for the E outputs
            b[0] = -(gy * v[5] - gz * v[4]);
            b[1] = -(gz * v[3] - gx * v[5]);
            b[2] = -(gx * v[4] - gy * v[3]);
            b[3] = gy * v[2] - gz * v[1];
            b[4] = gz * v[0] - gx * v[2];
            b[5] = gx * v[1] - gy * v[0];
        } else if (k < Kd) {
            const int j = k - 3 * Np;
#pragma unroll
            for (int f = 0; f < 6; ++f) b[f] = B[(RP + f * Nafp + j) * 16];
        } else {
#pragma unroll
            for (int f = 0; f < 6; ++f) b[f] = 0.f;
        }
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int f = 0; f < 6; ++f)
                acc[f][mt] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[mt], b[f], acc[f][mt], 0, 0, 0);
        __builtin_amdgcn_sched_barrier(0);
    }

    // ---- (4) fused low-storage RK update
    float *rt = A.res + (size_t)tile * (6 * Np * 64);
    float *ot = A.qout + (size_t)tile * (6 * Np * 64);
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) {
            const int n = 16 * mt + 4 * g + jj;
            if (n < Np) {
#pragma unroll
                for (int f = 0; f < 6; ++f) {
                    const unsigned idx = (unsigned)((f * Np + n) * 64 + col);
                    const float r = A.a * rt[idx] + A.dt * acc[f][mt][jj];
                    rt[idx] = r;
                    ot[idx] = B[(f * Np + n) * 16] + A.b * r;
                }
            }
        }
    }  // tile loop
}

template <int N>
static hipError_t launch3d(const StageArgs &a, hipStream_t s) {
    // every pointer the kernel dereferences must be set
    if (!a.opsfrag || !a.itab || !a.qin || !a.qout || !a.res || !a.geo || !a.fgeo || !a.nbr || a.ntiles <= 0 ||
        a.ngroups < 8 || (a.ngroups & 7))
        return hipErrorInvalidValue;
    hipLaunchKernelGGL((stage3d_kernel<N>), dim3(a.ngroups), dim3(256), 0, s, a);
    return hipGetLastError();
}

template <int N>
static int occupancy3d() {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, stage3d_kernel<N>, 256, 0) != hipSuccess) return 1;
    return nb > 0 ? nb : 1;
}

int blocks_per_cu_3d(int N) {
    switch (N) {
        case 1: return occupancy3d<1>();
        case 2: return occupancy3d<2>();
        case 3: return occupancy3d<3>();
        case 4: return occupancy3d<4>();
        default: return 1;
    }
}

hipError_t launch_stage3d(int N, const StageArgs &a, hipStream_t s) {
    switch (N) {
        case 1: return launch3d<1>(a, s);
        case 2: return launch3d<2>(a, s);
        case 3: return launch3d<3>(a, s);
        case 4: return launch3d<4>(a, s);
        default: return hipErrorInvalidValue;
    }
}

const char *stage3d_kernel_name(int N) {
    (void)N;
    return "stage3d_kernel<N>";
}

// Fragment-ordered copy of [Dr | Ds | Dt | LIFT] for the A operand:
// out[(mt*KS + ks)*64 + l] = Op[16 mt + l%16][4 ks + l/16].
int opsfrag3d(int N, const double *Dr, const double *Ds, const double *Dt, const double *LIFT, float *out) {
    const int Np = (N + 1) * (N + 2) * (N + 3) / 6, Nafp = 4 * ((N + 1) * (N + 2) / 2);
    const int Kd = 3 * Np + Nafp, KS = (Kd + 3) / 4, MT = (Np + 15) / 16;
    if (!out) return MT * KS * 64;
    for (int mt = 0; mt < MT; ++mt)
        for (int ks = 0; ks < KS; ++ks)
            for (int l = 0; l < 64; ++l) {
                const int row = 16 * mt + (l % 16), k = 4 * ks + l / 16;
                double v = 0.0;
                if (row < Np && k < Kd) {
                    if (k < Np)
                        v = Dr[row * Np + k];
                    else if (k < 2 * Np)
                        v = Ds[row * Np + (k - Np)];
                    else if (k < 3 * Np)
                        v = Dt[row * Np + (k - 2 * Np)];
                    else
                        v = LIFT[row * Nafp + (k - 3 * Np)];
                }
                out[(mt * KS + ks) * 64 + l] = (float)v;
            }
    return MT * KS * 64;
}

}  // namespace dgw
