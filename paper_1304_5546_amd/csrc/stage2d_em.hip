// Fused LSRK stage for 2D TM Maxwell, FP32, on the element-major field
// layout (the 2D counterpart of the 3D kernel's design).
//
// Per element and stage (eq. dg-strong-explicit):
//   1. reference derivatives Dr u, Ds u of each field u = Hx, Hy, Ez on the
//      matrix cores (v_mfma_f32_16x16x4_f32);
//   2. chain rule (eq. dg-diff-local-to-global) and the TM curl:
//      rhs_Hx = -d_y Ez / mu, rhs_Hy = d_x Ez / mu, rhs_Ez = (d_x Hy - d_y Hx) / eps;
//   3. the upwind flux at every face node (eq. max2d-numflux with the factor
//      1/2, [q] = q- - q+; exact Riemann flux across eps/mu jumps, blended by
//      alpha with the central flux), the partner trace through the face
//      record, on the PEC wall the mirror state E+ = -E-, H+ = H-;
//   4. rhs += LIFT flux on the matrix cores, then res <- a res + dt rhs,
//      q_out <- q_in + b res.
//
// Field layout [element][field][node], each field padded to NPP = Np rounded
// up to 4 nodes (pads hold 0).  A work unit is one wave and 16 elements (one
// MFMA N-tile, lane (g, c): element c).  Lane group g owns the nodes
// slot_node(KV, g, i), i < KV (runs of four consecutive nodes: one 16-byte
// access per lane and run).  The derivative operator is [Dr; Ds] packed by
// output slot (slot s = 4 mt + jj of lane group g holds D_(s mod 2) of node
// slot s / 2), its K rows follow the ownership (row 4 ks + g = node slot ks
// of lane group g); LIFT rows follow the ownership, its K rows are the face
// nodes.  So a lane finds both reference derivatives of its nodes in its own
// accumulators and updates exactly the nodes it loaded.  Each wave copies its
// elements' fields into LDS as they arrive; a work-group of WPG waves takes a
// window of WPG / 4 consecutive tiles, whose partner traces come from those
// LDS copies, the rest from memory (one contiguous block per partner,
// gathered SPD face nodes ahead).  Persistent grid, XCD-contiguous ranges.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "device.hpp"

namespace dgw {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

// waves per work-group: the LDS copies of 16 waves (4 tiles) fit up to order
// 7, of 8 waves (2 tiles) at order 8
__host__ __device__ constexpr int wpg_em(int N) { return N >= 8 ? 8 : 16; }

namespace {

template <int N, bool MAT>
struct TriE {
    static constexpr int Np = (N + 1) * (N + 2) / 2;
    static constexpr int Nfp = N + 1;
    static constexpr int Nafp = 3 * Nfp;
    static constexpr int NPP = npp_pad(Np);       // nodes per field in memory
    static constexpr int KV = NPP / 4;            // nodes per lane group
    static constexpr int NC = KV / 4;             // 16-byte runs per lane and field
    static constexpr int NR = KV - 4 * NC;        // single nodes per lane and field
    static constexpr int MTD = (2 * KV + 3) / 4;  // M-tiles of the packed [Dr; Ds]
    static constexpr int MTL = (KV + 3) / 4;      // M-tiles of LIFT
    static constexpr int KL = (Nafp + 3) / 4;     // K-steps of LIFT
    static constexpr int RS = 3 * NPP;            // floats per element
    // LDS stride of an element's copy: a multiple of 4 floats (16-byte
    // accesses) that is 4 mod 8, so the 16 elements of a lane group fall in 8
    // different bank quads
    static constexpr int ES = RS % 8 == 4 ? RS : RS + 4;
    static constexpr int NT = Nafp + 3 * 2 * Nfp; // face-node tables
    static constexpr int AV = MTD * KV * 64, AL = MTL * KL * 64;
    static constexpr int G = MAT ? 6 : 4;         // factor rows
    static constexpr int FG = MAT ? 6 : 3;        // face data rows per face
    static constexpr int WPG = wpg_em(N);
    static constexpr int TPW = WPG / 4;           // tiles per window
};

__device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc(const void *p, unsigned bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, (int)bytes, 0x00020000);
}
__device__ __forceinline__ float bload(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}
__device__ __forceinline__ void bstore(__amdgpu_buffer_rsrc_t r, float v, unsigned voff, unsigned soff) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, voff, soff, 0);
}
// 16-byte load into four floats (through a 128-bit integer: extracting the
// lanes of the vector result directly lets the compiler narrow the load)
__device__ __forceinline__ void bload4(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff, float *v) {
    const unsigned __int128 u = __builtin_bit_cast(unsigned __int128, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0));
#pragma unroll
    for (int k = 0; k < 4; ++k) v[k] = __builtin_bit_cast(float, (unsigned)(u >> (32 * k)));
}
__device__ __forceinline__ void bstore4(__amdgpu_buffer_rsrc_t r, const float *v, unsigned voff, unsigned soff) {
    u32x4 u;
#pragma unroll
    for (int k = 0; k < 4; ++k) u[k] = __builtin_bit_cast(unsigned, v[k]);
    __builtin_amdgcn_raw_buffer_store_b128(u, r, voff, soff, 0);
}

}  // namespace

#ifndef DGW_EM_SHARE
#define DGW_EM_SHARE 1  // partner traces inside the window from the other waves' LDS copies
#endif
#ifndef DGW_EM_SPD
#define DGW_EM_SPD 2  // face nodes of partner traces in flight ahead of their use
#endif

template <int N, bool MAT>
__global__ void __launch_bounds__(wpg_em(N) * 64) stage2d_em_kernel(StageArgs A) {
    using T = TriE<N, MAT>;
    constexpr int Np = T::Np, Nfp = T::Nfp, Nafp = T::Nafp, NPP = T::NPP, KV = T::KV, NC = T::NC, NR = T::NR;
    constexpr int MTD = T::MTD, MTL = T::MTL, KL = T::KL, RS = T::RS, ES = T::ES, NT = T::NT;
    constexpr int AV = T::AV, AL = T::AL, G = T::G, FG = T::FG, WPG = T::WPG, TPW = T::TPW;
    constexpr int FRAG4 = (AV + AL + 3) / 4;
    __shared__ uint4 sAq[FRAG4];
    __shared__ int stab[NT];
    __shared__ __attribute__((aligned(16))) float sF[WPG][16 * ES];
    const float *sA = reinterpret_cast<const float *>(sAq);

    {
        const uint4 *src = reinterpret_cast<const uint4 *>(A.opsfrag);
        for (int i = threadIdx.x; i < FRAG4; i += WPG * 64) sAq[i] = src[i];
        for (int i = threadIdx.x; i < NT; i += WPG * 64) stab[i] = A.itab[i];
    }
    __syncthreads();

    const int lane0 = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);

    // windows of TPW consecutive tiles (wave w: tile TPW p + w / 4, quarter
    // w % 4); each XCD walks a contiguous range of windows.  The loop bound
    // is uniform over the work-group (two barriers per window); a wave whose
    // tile lies past the mesh idles.
    const int nwin = (A.ntiles + TPW - 1) / TPW;
    const int x = blockIdx.x & 7, bi = blockIdx.x >> 3, GB = gridDim.x >> 3;
    const int q8 = nwin >> 3, r8 = nwin & 7;
    const int xbase = x * q8 + (x < r8 ? x : r8), xcount = q8 + (x < r8 ? 1 : 0);
    const float hs_alpha = 0.5f * A.alpha;

    float *F = sF[w];
    for (int pl = bi; pl < xcount; pl += GB) {
        const int win = xbase + pl;
        const int tile = TPW * win + (w >> 2);
        const bool active = tile < A.ntiles;  // wave-uniform
        int lane = lane0;
        asm volatile("" : "+v"(lane));
        const int g = lane >> 4, c = lane & 15;
        const int col = 16 * (w & 3) + c;
        constexpr unsigned TB = 64 * RS * 4;
        const __amdgpu_buffer_rsrc_t rq = rsrc(A.qin + (size_t)tile * (64 * RS), TB);
        const unsigned vel = (unsigned)(col * RS) * 4;
        const unsigned v16 = vel + 16u * (unsigned)g;
        const unsigned v4 = vel + 4u * (unsigned)g;
        float *Fc = F + c * ES;
        const unsigned vcol = (unsigned)col * 4;

        float cv[3][KV];
#pragma unroll
        for (int o = 0; o < 3; ++o)
#pragma unroll
            for (int i = 0; i < KV; ++i) cv[o][i] = 0.f;

        if (active) {
            // geometric factors with 1/mu (magnetic) and 1/eps (electric) folded in
            float Gf[G];
            {
                const __amdgpu_buffer_rsrc_t rg = rsrc(A.geo + (size_t)tile * (G * 64), G * 64 * 4);
#pragma unroll
                for (int q = 0; q < G; ++q) Gf[q] = bload(rg, vcol, q * 256);
            }
            const float ieps = MAT ? Gf[4 % G] : 1.f, imu = MAT ? Gf[5 % G] : 1.f;
            const float rx = Gf[0], ry = Gf[1], sx = Gf[2], sy = Gf[3];
            auto load_b = [&](int f, float (&b)[KV]) {
#pragma unroll
                for (int t = 0; t < NC; ++t) bload4(rq, v16, (f * NPP + 16 * t) * 4, &b[4 * t]);
#pragma unroll
                for (int r = 0; r < NR; ++r) b[4 * NC + r] = bload(rq, v4, (f * NPP + 16 * NC + 4 * r) * 4);
            };
            float bn[KV];
            load_b(0, bn);
            auto field = [&](auto FI) {
                constexpr int f = decltype(FI)::value;
                float b[KV];
#pragma unroll
                for (int i = 0; i < KV; ++i) b[i] = bn[i];
#pragma unroll
                for (int t = 0; t < NC; ++t)
                    *reinterpret_cast<floatx4 *>(Fc + f * NPP + 16 * t + 4 * g) =
                        floatx4{b[4 * t], b[4 * t + 1], b[4 * t + 2], b[4 * t + 3]};
#pragma unroll
                for (int r = 0; r < NR; ++r) Fc[f * NPP + 16 * NC + 4 * r + g] = b[4 * NC + r];
                if constexpr (f + 1 < 3) load_b(f + 1, bn);
                floatx4 d[MTD];
#pragma unroll
                for (int m = 0; m < MTD; ++m) d[m] = floatx4{0.f, 0.f, 0.f, 0.f};
                int la = lane;
                asm volatile("" : "+v"(la));
#pragma unroll
                for (int ks = 0; ks < KV; ++ks)
#pragma unroll
                    for (int m = 0; m < MTD; ++m)
                        d[m] = __builtin_amdgcn_mfma_f32_16x16x4f32(sA[(m * KV + ks) * 64 + la], b[ks], d[m], 0, 0, 0);
                // chain rule: slot 2 i + p holds D_p of node slot i; TM curl
#pragma unroll
                for (int i = 0; i < KV; ++i) {
                    const float dr = d[(2 * i) / 4][(2 * i) % 4], ds = d[(2 * i + 1) / 4][(2 * i + 1) % 4];
                    const float ux = rx * dr + sx * ds, uy = ry * dr + sy * ds;
                    if constexpr (f == 0) cv[2][i] -= ieps * uy;         // Ez -= d_y Hx / eps
                    if constexpr (f == 1) cv[2][i] += ieps * ux;         // Ez += d_x Hy / eps
                    if constexpr (f == 2) {
                        cv[0][i] -= imu * uy;                            // Hx -= d_y Ez / mu
                        cv[1][i] += imu * ux;                            // Hy += d_x Ez / mu
                    }
                }
#pragma unroll
                for (int o = 0; o < 3; ++o)
#pragma unroll
                    for (int i = 0; i < KV; ++i) asm volatile("" : "+v"(cv[o][i]));
                __builtin_amdgcn_sched_barrier(0);
            };
            field(std::integral_constant<int, 0>{});
            field(std::integral_constant<int, 1>{});
            field(std::integral_constant<int, 2>{});
        }  // active

        // ---- surface: face records of the element
        int rc0 = -1, rc1 = -1, rc2 = -1;
        if (active) {
            const __amdgpu_buffer_rsrc_t rn = rsrc(A.nbr + (size_t)tile * (3 * 64), 3 * 64 * 4);
            rc0 = __builtin_bit_cast(int, bload(rn, vcol, 0));
            rc1 = __builtin_bit_cast(int, bload(rn, vcol, 256));
            rc2 = __builtin_bit_cast(int, bload(rn, vcol, 512));
        }
        auto face_rec = [&](int face) { return face == 0 ? rc0 : face == 1 ? rc1 : rc2; };
        const __amdgpu_buffer_rsrc_t rall = rsrc(A.qin, (unsigned)A.ntiles * TB);
        struct Partner {
            int own, e2, pn;
            bool wall, inwin;
        };
        auto partner = [&](int j) {
            Partner P;
            const int jc = j < Nafp ? j : Nafp - 1;  // padding rows read a valid node
            const int face = jc / Nfp, i = jc - face * Nfp;
            P.own = stab[jc];
            const int rc = face_rec(face);
            P.wall = rc < 0;
            P.e2 = P.wall ? tile * 64 + col : (rc >> 5);
            P.pn = P.wall ? P.own : stab[Nafp + (((rc >> 3) & 3) * 2 + (rc & 7)) * Nfp + i];
            // with DGW_EM_SHARE = 0 a wave reads only its own LDS copy (its 16
            // elements) and runs without work-group barriers
            P.inwin = DGW_EM_SHARE ? (unsigned)((P.e2 >> 6) - TPW * win) < (unsigned)TPW
                                   : (P.e2 >> 4) == ((tile * 64 + col) >> 4);
            return P;
        };
        // partner traces outside the window, gathered SPD face nodes ahead
        auto gather = [&](int j, float (&pb)[3]) {
            const Partner P = partner(j);
            if (!P.inwin) {
                const unsigned vp = ((unsigned)P.e2 * RS + P.pn) * 4;
#pragma unroll
                for (int f = 0; f < 3; ++f) pb[f] = bload(rall, vp, f * NPP * 4);
            }
        };
        auto traces = [&](int j, const float (&pb)[3], float (&m)[3], float (&pv)[3]) {
            const Partner P = partner(j);
#pragma unroll
            for (int f = 0; f < 3; ++f) m[f] = Fc[f * NPP + P.own];
            if (P.inwin) {
                const int t2 = (P.e2 >> 6) - TPW * win;
                const float *F2 = sF[4 * t2 + ((P.e2 & 63) >> 4)] + (P.e2 & 15) * ES;
#pragma unroll
                for (int f = 0; f < 3; ++f) pv[f] = F2[f * NPP + P.pn];
            } else {
#pragma unroll
                for (int f = 0; f < 3; ++f) pv[f] = pb[f];
            }
            return P.wall;
        };
        constexpr int SPD = DGW_EM_SPD;
        float ring[SPD][3];
#pragma unroll
        for (int t = 0; t < SPD; ++t)
#pragma unroll
            for (int f = 0; f < 3; ++f) ring[t][f] = 0.f;
        if (active) {
#pragma unroll
            for (int t = 0; t < SPD; ++t)
                if (t < KL) gather(4 * t + g, ring[t]);
        }
        // every wave's LDS copy is complete: partner traces inside the window
        if (DGW_EM_SHARE) __syncthreads();
        if (active) {
            floatx4 acc[3][MTL];
#pragma unroll
            for (int o = 0; o < 3; ++o)
#pragma unroll
                for (int mt = 0; mt < MTL; ++mt)
#pragma unroll
                    for (int jj = 0; jj < 4; ++jj) {
                        constexpr int dummy = 0;
                        const int i = 4 * mt + jj;
                        acc[o][mt][jj] = i < KV ? cv[o][i < KV ? i : dummy] : 0.f;
                    }
            float fd[3 * FG];
            {
                const __amdgpu_buffer_rsrc_t rf = rsrc(A.fgeo + (size_t)tile * (3 * FG * 64), 3 * FG * 64 * 4);
#pragma unroll
                for (int q = 0; q < 3 * FG; ++q) fd[q] = bload(rf, vcol, q * 256);
            }
            auto face_val = [&](int face, int q) {
                return face == 0 ? fd[q] : face == 1 ? fd[FG + q] : fd[2 * FG + q];
            };
            // LIFT, K step ks: lane group g evaluates face node 4 ks + g
#pragma unroll
            for (int ks = 0; ks < KL; ++ks) {
                const int j = 4 * ks + g;
                float m[3], pv[3];
                const bool wall = traces(j, ring[ks % SPD], m, pv);
                if (ks + SPD < KL) gather(4 * (ks + SPD) + g, ring[ks % SPD]);
                const int face = (j < Nafp ? j : Nafp - 1) / Nfp;
                const float on = j < Nafp ? 1.f : 0.f;  // padding rows feed zero
                // [q] = q- - q+, with q+ = (H-, -E-) on the wall
                const float dHx = m[0] - pv[0], dHy = m[1] - pv[1];
                const float dEz = m[2] - (wall ? -pv[2] : pv[2]);
                const float nx = face_val(face, 0), ny = face_val(face, 1);
                const float dh = nx * dHy - ny * dHx;  // jump of the tangential field
                float cEE, cEh, cHE, cHh;
                if constexpr (MAT) {
                    cEE = face_val(face, 2);
                    cEh = face_val(face, 3 % FG);
                    cHE = face_val(face, 4 % FG);
                    cHh = face_val(face, 5 % FG);
                } else {
                    const float fs = face_val(face, 2);
                    cEE = hs_alpha * fs;
                    cEh = 0.5f * fs;
                    cHE = 0.5f * fs;
                    cHh = hs_alpha * fs;
                }
                const float fE = -(cEE * dEz + cEh * dh) * on;
                const float fH = (cHE * dEz + cHh * dh) * on;
                const float fl[3] = {ny * fH, -nx * fH, fE};
#pragma unroll
                for (int mt = 0; mt < MTL; ++mt) {
                    const float a = sA[AV + (mt * KL + ks) * 64 + lane];
#pragma unroll
                    for (int f = 0; f < 3; ++f)
                        acc[f][mt] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, fl[f], acc[f][mt], 0, 0, 0);
                }
                __builtin_amdgcn_sched_barrier(0);
            }

            // ---- fused low-storage RK update of the lane's nodes: every
            // residual load first, then per field the arithmetic and stores
            // (pad nodes carry zero rows: they stay 0)
            const __amdgpu_buffer_rsrc_t rr = rsrc(A.res + (size_t)tile * (64 * RS), TB);
            const __amdgpu_buffer_rsrc_t ro = rsrc(A.qout + (size_t)tile * (64 * RS), TB);
            float rv[3][KV];
#pragma unroll
            for (int f = 0; f < 3; ++f) {
#pragma unroll
                for (int t = 0; t < NC; ++t) bload4(rr, v16, (f * NPP + 16 * t) * 4, &rv[f][4 * t]);
#pragma unroll
                for (int r = 0; r < NR; ++r) rv[f][4 * NC + r] = bload(rr, v4, (f * NPP + 16 * NC + 4 * r) * 4);
            }
#pragma unroll
            for (int f = 0; f < 3; ++f) {
                float qv[KV];
#pragma unroll
                for (int t = 0; t < NC; ++t) {
                    const floatx4 q4 = *reinterpret_cast<const floatx4 *>(Fc + f * NPP + 16 * t + 4 * g);
#pragma unroll
                    for (int k = 0; k < 4; ++k) qv[4 * t + k] = q4[k];
                }
#pragma unroll
                for (int r = 0; r < NR; ++r) qv[4 * NC + r] = Fc[f * NPP + 16 * NC + 4 * r + g];
#pragma unroll
                for (int i = 0; i < KV; ++i) {
                    rv[f][i] = A.a * rv[f][i] + A.dt * acc[f][i / 4][i % 4];
                    qv[i] = qv[i] + A.b * rv[f][i];
                }
#pragma unroll
                for (int t = 0; t < NC; ++t) {
                    bstore4(rr, &rv[f][4 * t], v16, (f * NPP + 16 * t) * 4);
                    bstore4(ro, &qv[4 * t], v16, (f * NPP + 16 * t) * 4);
                }
#pragma unroll
                for (int r = 0; r < NR; ++r)
                    if (16 * NC + 4 * r + g < Np) {
                        bstore(rr, rv[f][4 * NC + r], v4, (f * NPP + 16 * NC + 4 * r) * 4);
                        bstore(ro, qv[4 * NC + r], v4, (f * NPP + 16 * NC + 4 * r) * 4);
                    }
            }
        }  // active
        if (DGW_EM_SHARE) __syncthreads();  // the LDS copies are read by other waves until here
    }
}

template <int N, bool MAT>
static hipError_t launch2d_em(const StageArgs &a, hipStream_t s) {
    if (!a.opsfrag || !a.itab || !a.qin || !a.qout || !a.res || !a.geo || !a.fgeo || !a.nbr || a.ntiles <= 0 ||
        a.ngroups < 8 || (a.ngroups & 7))
        return hipErrorInvalidValue;
    hipLaunchKernelGGL((stage2d_em_kernel<N, MAT>), dim3(a.ngroups), dim3(TriE<N, MAT>::WPG * 64), 0, s, a);
    return hipGetLastError();
}

template <int N, bool MAT>
static int occupancy2d_em() {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, stage2d_em_kernel<N, MAT>, TriE<N, MAT>::WPG * 64, 0) !=
        hipSuccess)
        return 1;
    return nb > 0 ? nb : 1;
}

hipError_t launch_stage2d_em(int N, bool material, const StageArgs &a, hipStream_t s) {
    switch (N) {
        case 1: return material ? launch2d_em<1, true>(a, s) : launch2d_em<1, false>(a, s);
        case 2: return material ? launch2d_em<2, true>(a, s) : launch2d_em<2, false>(a, s);
        case 3: return material ? launch2d_em<3, true>(a, s) : launch2d_em<3, false>(a, s);
        case 4: return material ? launch2d_em<4, true>(a, s) : launch2d_em<4, false>(a, s);
        case 5: return material ? launch2d_em<5, true>(a, s) : launch2d_em<5, false>(a, s);
        case 6: return material ? launch2d_em<6, true>(a, s) : launch2d_em<6, false>(a, s);
        case 7: return material ? launch2d_em<7, true>(a, s) : launch2d_em<7, false>(a, s);
        case 8: return material ? launch2d_em<8, true>(a, s) : launch2d_em<8, false>(a, s);
        default: return hipErrorInvalidValue;
    }
}

int blocks_per_cu_2d_em(int N, bool material) {
    switch (N) {
        case 1: return material ? occupancy2d_em<1, true>() : occupancy2d_em<1, false>();
        case 2: return material ? occupancy2d_em<2, true>() : occupancy2d_em<2, false>();
        case 3: return material ? occupancy2d_em<3, true>() : occupancy2d_em<3, false>();
        case 4: return material ? occupancy2d_em<4, true>() : occupancy2d_em<4, false>();
        case 5: return material ? occupancy2d_em<5, true>() : occupancy2d_em<5, false>();
        case 6: return material ? occupancy2d_em<6, true>() : occupancy2d_em<6, false>();
        case 7: return material ? occupancy2d_em<7, true>() : occupancy2d_em<7, false>();
        case 8: return material ? occupancy2d_em<8, true>() : occupancy2d_em<8, false>();
        default: return 1;
    }
}

// Work-groups of the persistent grid walk windows of this many tiles.
int tiles_per_group_2d_em(int N) { return wpg_em(N) / 4; }

// A-fragment order of the element-major 2D kernel's operators: the packed
// derivative operator, out[(mt*KV + ks)*64 + l] = row (mt, l % 16), K row
// 4 ks + l / 16 (= node slot_node(KV, l / 16, ks)), then LIFT,
// out[AV + (mt*KL + ks)*64 + l] = row (mt, l % 16), face node 4 ks + l / 16.
// Row r of M-tile mt is output slot 4 mt + r % 4 of lane group r / 4.
// Returns the number of floats.
int opsfrag2d_em(int N, const double *Dr, const double *Ds, const double *LIFT, float *out) {
    const int Np = (N + 1) * (N + 2) / 2, Nafp = 3 * (N + 1), KV = npp_pad(Np) / 4;
    const int MTD = (2 * KV + 3) / 4, MTL = (KV + 3) / 4, KL = (Nafp + 3) / 4;
    const int AV = MTD * KV * 64, AL = MTL * KL * 64;
    if (!out) return AV + AL;
    const double *D[2] = {Dr, Ds};
    for (int mt = 0; mt < MTD; ++mt)
        for (int ks = 0; ks < KV; ++ks)
            for (int l = 0; l < 64; ++l) {
                const int r = l % 16, g = r / 4, s = 4 * mt + r % 4;
                const int ni = slot_node(KV, l / 16, ks);
                double v = 0.0;
                if (s < 2 * KV) {
                    const int no = slot_node(KV, g, s / 2);
                    if (no < Np && ni < Np) v = D[s % 2][(size_t)no * Np + ni];
                }
                out[(mt * KV + ks) * 64 + l] = (float)v;
            }
    for (int mt = 0; mt < MTL; ++mt)
        for (int ks = 0; ks < KL; ++ks)
            for (int l = 0; l < 64; ++l) {
                const int r = l % 16, g = r / 4, s = 4 * mt + r % 4, j = 4 * ks + l / 16;
                double v = 0.0;
                if (s < KV) {
                    const int no = slot_node(KV, g, s);
                    if (no < Np && j < Nafp) v = LIFT[(size_t)no * Nafp + j];
                }
                out[AV + (mt * KL + ks) * 64 + l] = (float)v;
            }
    return AV + AL;
}

}  // namespace dgw
