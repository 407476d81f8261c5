// Fused LSRK stage for 3D Maxwell on tetrahedra (eps = mu = 1), FP32, with
// the element-local contractions on the matrix cores (v_mfma_f32_16x16x4_f32).
//
// 3D analogue of eq. dg-strong-explicit (section "Adding Generality": the
// kernels change only mildly).  Per element and stage:
//   1. reference derivatives D_p u (p = r, s, t) of each of the six fields u
//      (MFMA: [Dr; Ds; Dt] against the field's nodal values);
//   2. chain rule and curl on those derivatives (eq. dg-diff-local-to-global,
//      g_p = grad p constant per affine element):
//        rhs_H = -curl E,  rhs_E = curl H,  d_x u = sum_p (p_x) D_p u, ...;
//   3. upwind flux at every face node (3D form of eq. max2d-numflux, factor
//      1/2, [q] = q- - q+):
//        flux_H = Fscale/2 ( n x [E] + alpha (n (n.[H]) - [H]) )
//        flux_E = Fscale/2 (-n x [H] + alpha (n (n.[E]) - [E]) ),
//      the partner trace through the face record and the orientation table,
//      on the PEC wall the mirror state E+ = -E-, H+ = H-;
//   4. rhs += LIFT flux (MFMA), then res <- a res + dt rhs,
//      q_out <- q_in + b res.
//
// Work unit = one wave and 16 consecutive elements (one MFMA N-tile; lane
// (g, c) = (lane / 16, lane % 16) works on element column c).  The operands
// of the derivatives are read straight from HBM (buffer loads sharing one
// address register per lane): the B fragment of K-step ks is rows 4 ks + g
// of the field, a 64-byte piece of each of four 256-byte rows; the eight
// waves of a work-group take the quarters of two 64-element tiles together.
// As they arrive the values are also written to the wave's LDS copy of its
// elements' fields, from which the face traces and the update read them (no
// second trip to memory).  The LDS also holds the operator fragments and the
// face-node tables.  Persistent grid with XCD-contiguous ranges of tiles.
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
    static constexpr int MT = (Np + 15) / 16;   // M-tiles of the output nodes
    static constexpr int KV = (Np + 3) / 4;     // K-steps of a derivative
    static constexpr int KL = (Nafp + 3) / 4;   // K-steps of LIFT
    static constexpr int AV = 3 * MT * KV * 64; // derivative fragments (floats)
    static constexpr int AL = MT * KL * 64;     // LIFT fragments
    static constexpr int NT = Nafp + 4 * 6 * Nfp;  // face-node tables
};

// Buffer resource over `bytes` bytes at a wave-uniform base: loads through it
// take one per-lane 32-bit offset plus a scalar offset (the row), so rows of
// a tile share one address register; accesses past `bytes` read 0 / drop.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc(const void *p, unsigned bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, (int)bytes, 0x00020000);
}
__device__ __forceinline__ float bload(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}
__device__ __forceinline__ void bstore(__amdgpu_buffer_rsrc_t r, float v, unsigned voff, unsigned soff) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, voff, soff, 0);
}

}  // namespace

// Tuning: K-steps of face traces kept in flight, fields of volume operands
// kept in flight.  One K-step of traces keeps the kernel within its 256
// registers; with two, registers spill to scratch and the order-4 stage runs
// 14 % slower.
#ifndef DGW_3D_SPD
#define DGW_3D_SPD 1
#endif
#ifndef DGW_3D_VPD
#define DGW_3D_VPD 1
#endif
constexpr int SPD = DGW_3D_SPD;
constexpr int VPD = DGW_3D_VPD;

template <int N>
__global__ void __launch_bounds__(512) stage3d_kernel(StageArgs A) {
    using T = Tet<N>;
    constexpr int Np = T::Np, Nfp = T::Nfp, Nafp = T::Nafp, MT = T::MT, KV = T::KV, KL = T::KL;
    constexpr int AV = T::AV, AL = T::AL, NT = T::NT;
    __shared__ float sA[AV + AL];
    __shared__ int stab[NT];
    // each wave's copy of its 16 elements' fields, [field * Np + node][17]
    // (row stride 17: rows of different lane groups fall in different banks);
    // the face traces and the update read the element's own values here
    // instead of from memory again
    constexpr int FS = 17;
    __shared__ float sF[8][6 * Np * FS];

    for (int i = threadIdx.x; i < AV + AL; i += 512) sA[i] = A.opsfrag[i];
    for (int i = threadIdx.x; i < NT; i += 512) stab[i] = A.itab[i];
    __syncthreads();

    const int lane0 = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);

    // the work-group takes two consecutive tiles at a time (wave w: tile
    // 2 p + w / 4, quarter w % 4); each XCD walks a contiguous range of tile
    // pairs.  The loop bound is uniform over the work-group (it meets two
    // barriers per pair); a wave whose tile lies past the mesh idles.
    const int npairs = (A.ntiles + 1) >> 1;
    const int x = blockIdx.x & 7, bi = blockIdx.x >> 3, GB = gridDim.x >> 3;
    const int q8 = npairs >> 3, r8 = npairs & 7;
    const int xbase = x * q8 + (x < r8 ? x : r8), xcount = q8 + (x < r8 ? 1 : 0);
    const float ha = 0.5f * A.alpha;

    float *F = sF[w];
    for (int pl = bi; pl < xcount; pl += GB) {
        const int pair = xbase + pl;
        const int tile = 2 * pair + (w >> 2);
        const bool active = tile < A.ntiles;  // wave-uniform
        // lane indices opaque to the compiler: per-lane offsets are recomputed
        // per work unit rather than hoisted into long-lived registers
        int lane = lane0;
        asm volatile("" : "+v"(lane));
        const int g = lane >> 4, c = lane & 15;
        const int col = 16 * (w & 3) + c;
        constexpr unsigned TB = 6 * Np * 64 * 4;  // bytes of a tile's fields
        const __amdgpu_buffer_rsrc_t rq = rsrc(A.qin + (size_t)tile * (6 * Np * 64), TB);
        const unsigned vcol = (unsigned)col * 4;             // column within a row
        const unsigned vrow = (unsigned)(g * 64 + col) * 4;  // row 4 ks + g of a K-step

        float G[9];
        float cv[6][MT][4];
        if (active) {
        {
            const __amdgpu_buffer_rsrc_t rg = rsrc(A.geo + (size_t)tile * (9 * 64), 9 * 64 * 4);
#pragma unroll
            for (int q = 0; q < 9; ++q) G[q] = bload(rg, vcol, q * 256);
        }

        // volume part of the right-hand side, in plain registers
#pragma unroll
        for (int f = 0; f < 6; ++f)
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                for (int jj = 0; jj < 4; ++jj) cv[f][mt][jj] = 0.f;

        // ---- volume: derivatives of field f, then their curl contributions
        // operands of the next VPD fields in flight (a ring of registers);
        // rows past Np belong to the next field (or lie past the tile, read
        // as 0): their operator columns are zero, so they need no masking
        float bring[VPD][KV];
#pragma unroll
        for (int f0 = 0; f0 < VPD; ++f0)
#pragma unroll
            for (int ks = 0; ks < KV; ++ks) bring[f0][ks] = bload(rq, vrow, (f0 * Np + 4 * ks) * 256);
#pragma unroll
        for (int f = 0; f < 6; ++f) {
            float bq[KV];
#pragma unroll
            for (int ks = 0; ks < KV; ++ks) {
                bq[ks] = bring[f % VPD][ks];
                if (4 * ks + g < Np) F[(f * Np + 4 * ks + g) * FS + c] = bq[ks];
            }
            if (f + VPD < 6) {
#pragma unroll
                for (int ks = 0; ks < KV; ++ks) bring[f % VPD][ks] = bload(rq, vrow, ((f + VPD) * Np + 4 * ks) * 256);
            }
            floatx4 d[3][MT];
#pragma unroll
            for (int p = 0; p < 3; ++p)
#pragma unroll
                for (int mt = 0; mt < MT; ++mt) d[p][mt] = floatx4{0.f, 0.f, 0.f, 0.f};
            // the operator fragments are re-read from LDS for every field: an
            // index opaque to the compiler keeps it from holding all of them
            // in registers across the six fields
            int la = lane;
            asm volatile("" : "+v"(la));
#pragma unroll
            for (int ks = 0; ks < KV; ++ks)
#pragma unroll
                for (int p = 0; p < 3; ++p)
#pragma unroll
                    for (int mt = 0; mt < MT; ++mt)
                        d[p][mt] = __builtin_amdgcn_mfma_f32_16x16x4f32(sA[((p * MT + mt) * KV + ks) * 64 + la],
                                                                       bq[ks], d[p][mt], 0, 0, 0);
            // chain rule: d_x u = r_x D_r u + s_x D_s u + t_x D_t u, ...
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                for (int jj = 0; jj < 4; ++jj) {
                    const float dr = d[0][mt][jj], ds = d[1][mt][jj], dtt = d[2][mt][jj];
                    const float gx = G[0] * dr + G[3] * ds + G[6] * dtt;
                    const float gy = G[1] * dr + G[4] * ds + G[7] * dtt;
                    const float gz = G[2] * dr + G[5] * ds + G[8] * dtt;
                    // fields 0..5 = Hx, Hy, Hz, Ex, Ey, Ez
                    if (f == 0) { cv[4][mt][jj] += gz; cv[5][mt][jj] -= gy; }  // Ey += dz Hx, Ez -= dy Hx
                    if (f == 1) { cv[3][mt][jj] -= gz; cv[5][mt][jj] += gx; }  // Ex -= dz Hy, Ez += dx Hy
                    if (f == 2) { cv[3][mt][jj] += gy; cv[4][mt][jj] -= gx; }  // Ex += dy Hz, Ey -= dx Hz
                    if (f == 3) { cv[1][mt][jj] -= gz; cv[2][mt][jj] += gy; }  // Hy -= dz Ex, Hz += dy Ex
                    if (f == 4) { cv[0][mt][jj] += gz; cv[2][mt][jj] -= gx; }  // Hx += dz Ey, Hz -= dx Ey
                    if (f == 5) { cv[0][mt][jj] -= gy; cv[1][mt][jj] += gx; }  // Hx -= dy Ez, Hy += dx Ez
                }
            // materialise the sums here: otherwise they are sunk to their use
            // in the update and every field's derivatives stay live until then
#pragma unroll
            for (int o = 0; o < 6; ++o)
#pragma unroll
                for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                    for (int jj = 0; jj < 4; ++jj) asm volatile("" : "+v"(cv[o][mt][jj]));
            __builtin_amdgcn_sched_barrier(0);
        }
        }  // active
        // every wave's LDS copy of its fields is complete: partner traces of
        // elements in this pair of tiles are read from there
        __syncthreads();
        if (active) {

        // ---- surface: flux at face node j = 4 ks + g, then LIFT.  The face
        // records and face data of the element are loaded once, up front, and
        // held as scalars (selected per lane, no per-lane array indexing): a
        // load whose value is needed in the same step would make the step
        // wait for every load issued before it, prefetched traces included
        const __amdgpu_buffer_rsrc_t rn = rsrc(A.nbr + (size_t)tile * (4 * 64), 4 * 64 * 4);
        const __amdgpu_buffer_rsrc_t rf = rsrc(A.fgeo + (size_t)tile * (16 * 64), 16 * 64 * 4);
        const int rc0 = __builtin_bit_cast(int, bload(rn, vcol, 0)), rc1 = __builtin_bit_cast(int, bload(rn, vcol, 256));
        const int rc2 = __builtin_bit_cast(int, bload(rn, vcol, 512)), rc3 = __builtin_bit_cast(int, bload(rn, vcol, 768));
        float fd[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) fd[q] = bload(rf, vcol, q * 256);
        auto face_rec = [&](int face) { return face == 0 ? rc0 : face == 1 ? rc1 : face == 2 ? rc2 : rc3; };
        auto face_val = [&](int face, int q) {
            return face == 0 ? fd[q] : face == 1 ? fd[4 + q] : face == 2 ? fd[8 + q] : fd[12 + q];
        };
        // all partner traces through one resource over the field array
        const __amdgpu_buffer_rsrc_t rall = rsrc(A.qin, (unsigned)A.ntiles * TB);
        // own and partner traces of face node j (on the wall the partner is
        // the element itself; the mirror sign is applied with the jump)
        auto load_traces = [&](int ks, float (&m)[6], float (&pv)[6], int &wall) {
            const int j = 4 * ks + g;
            const int jc = j < Nafp ? j : Nafp - 1;  // lanes past the faces read a valid node
            const int face = jc / Nfp, i = jc - face * Nfp;
            const int own = stab[jc];
            const int rc = face_rec(face);
            wall = rc < 0;
            const int e2 = wall ? tile * 64 + col : (rc >> 5);
            const int pn = wall ? own : stab[Nafp + (((rc >> 3) & 3) * 6 + (rc & 7)) * Nfp + i];
            const unsigned vp = (((unsigned)(e2 >> 6) * (6 * Np) + pn) * 64 + (e2 & 63)) * 4;
            const int t2 = (e2 >> 6) - 2 * pair;  // partner tile within the pair?
#pragma unroll
            for (int f = 0; f < 6; ++f) m[f] = F[(f * Np + own) * FS + c];
            if ((unsigned)t2 < 2u) {
                const float *F2 = sF[4 * t2 + ((e2 & 63) >> 4)];
#pragma unroll
                for (int f = 0; f < 6; ++f) pv[f] = F2[(f * Np + pn) * FS + (e2 & 15)];
            } else {
#pragma unroll
                for (int f = 0; f < 6; ++f) pv[f] = bload(rall, vp, f * Np * 256);
            }
        };
        // the LIFT contraction accumulates on top of the volume part
        floatx4 acc[6][MT];
#pragma unroll
        for (int f = 0; f < 6; ++f)
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
                acc[f][mt] = floatx4{cv[f][mt][0], cv[f][mt][1], cv[f][mt][2], cv[f][mt][3]};
        // traces of the next SPD K-steps in flight (a ring of registers)
        float mb[SPD][6], pb[SPD][6];
        int wb[SPD];
#pragma unroll
        for (int s0 = 0; s0 < SPD; ++s0)
            if (s0 < KL) load_traces(s0, mb[s0], pb[s0], wb[s0]);
#pragma unroll
        for (int ks = 0; ks < KL; ++ks) {
            float m[6], pv[6];
            const int slot = ks % SPD;
#pragma unroll
            for (int f = 0; f < 6; ++f) {
                m[f] = mb[slot][f];
                pv[f] = pb[slot][f];
            }
            const int wall = wb[slot];
            if (ks + SPD < KL) load_traces(ks + SPD, mb[slot], pb[slot], wb[slot]);
            const int j = 4 * ks + g;
            const int face = (j < Nafp ? j : Nafp - 1) / Nfp;
            // [q] = q- - q+, with q+ = (H-, -E-) on the wall
            float d[6];
#pragma unroll
            for (int f = 0; f < 6; ++f) d[f] = m[f] - ((wall && f >= 3) ? -pv[f] : pv[f]);
            const float nx = face_val(face, 0), ny = face_val(face, 1);
            const float nz = face_val(face, 2), fs = face_val(face, 3);
            const float dHx = d[0], dHy = d[1], dHz = d[2], dEx = d[3], dEy = d[4], dEz = d[5];
            const float ndH = nx * dHx + ny * dHy + nz * dHz;
            const float ndE = nx * dEx + ny * dEy + nz * dEz;
            const float h = j < Nafp ? 0.5f * fs : 0.f, ah = j < Nafp ? ha * fs : 0.f;
            const float cEx = ny * dEz - nz * dEy, cEy = nz * dEx - nx * dEz, cEz = nx * dEy - ny * dEx;
            const float cHx = ny * dHz - nz * dHy, cHy = nz * dHx - nx * dHz, cHz = nx * dHy - ny * dHx;
            float fl[6];
            fl[0] = h * cEx + ah * (nx * ndH - dHx);
            fl[1] = h * cEy + ah * (ny * ndH - dHy);
            fl[2] = h * cEz + ah * (nz * ndH - dHz);
            fl[3] = -h * cHx + ah * (nx * ndE - dEx);
            fl[4] = -h * cHy + ah * (ny * ndE - dEy);
            fl[5] = -h * cHz + ah * (nz * ndE - dEz);
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) {
                const float a = sA[AV + (mt * KL + ks) * 64 + lane];
#pragma unroll
                for (int f = 0; f < 6; ++f) acc[f][mt] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, fl[f], acc[f][mt], 0, 0, 0);
            }
            __builtin_amdgcn_sched_barrier(0);
        }

        // ---- fused low-storage RK update
        const __amdgpu_buffer_rsrc_t rr = rsrc(A.res + (size_t)tile * (6 * Np * 64), TB);
        const __amdgpu_buffer_rsrc_t ro = rsrc(A.qout + (size_t)tile * (6 * Np * 64), TB);
        const unsigned vout = (unsigned)(4 * g * 64 + col) * 4;  // row 16 mt + 4 g + jj
        // per field: all loads, then all arithmetic, then the stores (a store
        // between two loads orders them and exposes one memory latency per
        // value).  Rows 16 mt + 4 g + jj >= Np read the next field's rows (or
        // 0 past the tile) and are not stored.
#pragma unroll
        for (int f = 0; f < 6; ++f) {
            float rv[MT][4], qv[MT][4];
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                for (int jj = 0; jj < 4; ++jj) {
                    const unsigned so = (f * Np + 16 * mt + jj) * 256;
                    rv[mt][jj] = bload(rr, vout, so);
                    const int n = 16 * mt + 4 * g + jj;
                    qv[mt][jj] = n < Np ? F[(f * Np + n) * FS + c] : 0.f;
                }
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                for (int jj = 0; jj < 4; ++jj) {
                    rv[mt][jj] = A.a * rv[mt][jj] + A.dt * acc[f][mt][jj];
                    qv[mt][jj] = qv[mt][jj] + A.b * rv[mt][jj];
                }
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                for (int jj = 0; jj < 4; ++jj) {
                    if (16 * mt + 4 * g + jj < Np) {
                        const unsigned so = (f * Np + 16 * mt + jj) * 256;
                        bstore(rr, rv[mt][jj], vout, so);
                        bstore(ro, qv[mt][jj], vout, so);
                    }
                }
        }
        }  // active
        __syncthreads();  // the LDS copies are read by other waves until here
    }
}

template <int N>
static hipError_t launch3d(const StageArgs &a, hipStream_t s) {
    // every pointer the kernel dereferences must be set
    if (!a.opsfrag || !a.itab || !a.qin || !a.qout || !a.res || !a.geo || !a.fgeo || !a.nbr || a.ntiles <= 0 ||
        a.ngroups < 8 || (a.ngroups & 7))
        return hipErrorInvalidValue;
    hipLaunchKernelGGL((stage3d_kernel<N>), dim3(a.ngroups), dim3(512), 0, s, a);
    return hipGetLastError();
}

template <int N>
static int occupancy3d() {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, stage3d_kernel<N>, 512, 0) != hipSuccess) return 1;
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

// A-fragment order of the 3D kernel's operators: first Dr, Ds, Dt
// (out[((p*MT + mt)*KV + ks)*64 + l] = D_p[16 mt + l%16][4 ks + l/16]), then
// LIFT (out[AV + (mt*KL + ks)*64 + l] = LIFT[16 mt + l%16][4 ks + l/16]);
// zero outside the matrices.  Returns the number of floats.
int opsfrag3d(int N, const double *Dr, const double *Ds, const double *Dt, const double *LIFT, float *out) {
    const int Np = (N + 1) * (N + 2) * (N + 3) / 6, Nafp = 4 * ((N + 1) * (N + 2) / 2);
    const int MT = (Np + 15) / 16, KV = (Np + 3) / 4, KL = (Nafp + 3) / 4;
    const int AV = 3 * MT * KV * 64, AL = MT * KL * 64;
    if (!out) return AV + AL;
    const double *D[3] = {Dr, Ds, Dt};
    for (int p = 0; p < 3; ++p)
        for (int mt = 0; mt < MT; ++mt)
            for (int ks = 0; ks < KV; ++ks)
                for (int l = 0; l < 64; ++l) {
                    const int row = 16 * mt + (l % 16), k = 4 * ks + l / 16;
                    out[((p * MT + mt) * KV + ks) * 64 + l] = (row < Np && k < Np) ? (float)D[p][row * Np + k] : 0.f;
                }
    for (int mt = 0; mt < MT; ++mt)
        for (int ks = 0; ks < KL; ++ks)
            for (int l = 0; l < 64; ++l) {
                const int row = 16 * mt + (l % 16), k = 4 * ks + l / 16;
                out[AV + (mt * KL + ks) * 64 + l] = (row < Np && k < Nafp) ? (float)LIFT[row * Nafp + k] : 0.f;
            }
    return AV + AL;
}

}  // namespace dgw
