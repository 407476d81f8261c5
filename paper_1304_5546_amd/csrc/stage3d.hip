// Fused LSRK stage for 3D Maxwell on tetrahedra (eps = mu = 1), with the
// element-local contractions on the matrix cores: FP32 products
// (v_mfma_f32_16x16x4_f32) or split-BF16 products
// (v_mfma_f32_16x16x32_bf16, Op b = Op_hi b_hi + Op_hi b_lo + Op_lo b_hi,
// x_hi = bf16(x), x_lo = bf16(x - x_hi), FP32 accumulation).
//
// 3D analogue of eq. dg-strong-explicit (section "Adding Generality": the
// kernels change only mildly).  Per element and stage:
//   1. reference derivatives D_p u (p = r, s, t) of each of the six fields u;
//   2. chain rule and curl on those derivatives (eq. dg-diff-local-to-global,
//      g_p = grad p constant per affine element):
//        rhs_H = -curl E,  rhs_E = curl H,  d_x u = sum_p (p_x) D_p u, ...;
//   3. upwind flux at every face node (3D form of eq. max2d-numflux, factor
//      1/2, [q] = q- - q+):
//        flux_H = Fscale/2 ( n x [E] + alpha (n (n.[H]) - [H]) )
//        flux_E = Fscale/2 (-n x [H] + alpha (n (n.[E]) - [E]) ),
//      the partner trace through the face record and the orientation table,
//      on the PEC wall the mirror state E+ = -E-, H+ = H-;
//   4. rhs += LIFT flux, then res <- a res + dt rhs, q_out <- q_in + b res.
// The split form keeps the geometric factors, normals and Fscale in FP64:
// the chain rule and the flux are evaluated in FP64 and rounded to FP32 once;
// its derivative operand is u - u(node 0) (D_p annihilates constants, so the
// split carries the variation of u across the element, not its mean).
//
// Field layout: element-major, [element][field][node] with each field padded
// to NPP = Np rounded up to 4 nodes.  A work unit is one wave and 16
// elements (one MFMA N-tile, lane (g, c) = (lane / 16, lane % 16) works on
// element c).  Lane group g owns the nodes slot_node(KV, g, i), i < KV:
// runs of four consecutive nodes, so operands, residual and new fields move
// as one 16-byte access per lane and run.  The output rows of every
// contraction are permuted to the same ownership, so the accumulators of a
// lane hold exactly the nodes it loads and stores:
//   - the FP32 derivative operator is [Dr; Ds; Dt] packed by output slot:
//     slot s = 4 mt + jj of lane group g holds D_(s mod 3) of node
//     slot_node(KV, g, s / 3), so one lane finds the three reference
//     derivatives of a node in its own registers (7 M-tiles at order 4
//     instead of 3 x 3); its K rows follow the same ownership (row 4 ks + g
//     is node slot_node(KV, g, ks));
//   - the split derivative operator has the same rows, K rows in node order
//     (lane group g holds K rows 32 ks + 8 g .. + 7: two 16-byte runs);
//   - LIFT rows follow the ownership (slot 4 mt + jj = node slot i), its K
//     rows are the face nodes in face order.
// The wave copies its elements' fields into LDS as they arrive; face traces
// and the update read them there.  A work-group (8 waves) takes a pair of
// 64-element tiles: partner traces inside the pair come from the other
// waves' LDS copies, the rest from memory (one contiguous element block per
// partner).  Persistent grid with XCD-contiguous ranges of tile pairs.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "device.hpp"

namespace dgw {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float float2v __attribute__((ext_vector_type(2)));
typedef short shortx4 __attribute__((ext_vector_type(4)));

namespace {

template <int N>
struct Tet {
    static constexpr int Np = (N + 1) * (N + 2) * (N + 3) / 6;
    static constexpr int Nfp = (N + 1) * (N + 2) / 2;
    static constexpr int Nafp = 4 * Nfp;
    static constexpr int NPP = npp_pad(Np);        // nodes per field in memory
    static constexpr int KV = NPP / 4;           // nodes per lane group
    static constexpr int NC = KV / 4;            // 16-byte runs per lane and field
    static constexpr int NR = KV - 4 * NC;       // single nodes per lane and field
    static constexpr int MTD = (3 * KV + 3) / 4; // M-tiles of the packed derivative operator
    static constexpr int MTL = (KV + 3) / 4;     // M-tiles of LIFT
    static constexpr int KL = (Nafp + 3) / 4;    // K-steps of LIFT, FP32
    // split derivative: 16-bit K steps of 32 nodes; when at least one is full
    // and at most 8 nodes remain, those are contracted in FP32 (KT K steps of
    // 4) instead of a mostly empty 16-bit step
    static constexpr int TAILN = NPP % 32;
    static constexpr bool TAIL = NPP >= 32 && TAILN > 0 && TAILN <= 8;
    static constexpr int KVS = TAIL ? NPP / 32 : (NPP + 31) / 32;  // 16-bit K steps of a derivative
    static constexpr int KT = TAIL ? TAILN / 4 : 0;                 // FP32 K steps of its tail
    static constexpr int KLS = (Nafp + 15) / 16; // K-steps of LIFT, split (16-bit products of K 16)
    static constexpr int RS = 6 * NPP;           // floats per element
    // LDS stride of an element's copy: a multiple of 4 floats (16-byte
    // accesses) that is 4 mod 8, so the 16 elements of a lane group fall in 8
    // different bank quads
    static constexpr int ES = RS % 8 == 4 ? RS : RS + 4;
    static constexpr int NT = Nafp + 4 * 6 * Nfp;
    // operator fragments: FP32 floats (derivative, then LIFT); split uint4
    // (8 BF16) hi parts (derivative, LIFT) then lo parts
    static constexpr int AV = MTD * KV * 64, AL = MTL * KL * 64;
    // split: derivative fragments FV (uint4 = 8 BF16 per lane) hi then lo,
    // LIFT fragments FL (uint2 = 4 BF16 per lane) hi then lo
    static constexpr int FV = MTD * KVS * 64, FL = MTL * KLS * 64;
    static constexpr int FT = MTD * KT * 64;  // FP32 tail fragments (floats), after the lo parts
    static_assert(16 * NC <= Np, "a 16-byte run holds no pad node");
};

// Buffer resource over `bytes` bytes at a wave-uniform base: loads through it
// take one per-lane 32-bit offset plus a scalar offset, so the runs and
// fields of an element share one address register per lane; accesses past
// `bytes` read 0 / drop.
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
__device__ __forceinline__ floatx4 mfma3(bf16x8 ah, bf16x8 al, bf16x8 bh, bf16x8 bl, floatx4 c) {
    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl, c, 0, 0, 0);
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh, c, 0, 0, 0);
}
__device__ __forceinline__ bf16x8 as_bf16x8(uint4 u) {
    bf16x8 v;
    __builtin_memcpy(&v, &u, 16);
    return v;
}

// Curl contributions of the derivatives (gx, gy, gz) of field f (0..5 =
// Hx, Hy, Hz, Ex, Ey, Ez) to the right-hand sides: rhs_H = -curl E,
// rhs_E = curl H.
template <int F, typename V>
__device__ __forceinline__ void curl_add(V gx, V gy, V gz, float &o0, float &o1, float &o2, float &o3, float &o4,
                                         float &o5) {
    if constexpr (F == 0) { o4 += (float)gz; o5 -= (float)gy; }  // Ey += dz Hx, Ez -= dy Hx
    if constexpr (F == 1) { o3 -= (float)gz; o5 += (float)gx; }  // Ex -= dz Hy, Ez += dx Hy
    if constexpr (F == 2) { o3 += (float)gy; o4 -= (float)gx; }  // Ex += dy Hz, Ey -= dx Hz
    if constexpr (F == 3) { o1 -= (float)gz; o2 += (float)gy; }  // Hy -= dz Ex, Hz += dy Ex
    if constexpr (F == 4) { o0 += (float)gz; o2 -= (float)gx; }  // Hx += dz Ey, Hz -= dx Ey
    if constexpr (F == 5) { o0 -= (float)gy; o1 += (float)gx; }  // Hx -= dy Ez, Hy += dx Ez
}

// Flux of one face node from the jump d = q- - q+ (6 fields), the outward
// normal and Fscale (h = Fscale/2, ah = alpha Fscale/2; both 0 on padding
// rows).  R = float or double.
template <typename R>
__device__ __forceinline__ void face_flux(const R (&d)[6], R nx, R ny, R nz, R h, R ah, R (&fl)[6]) {
    const R dHx = d[0], dHy = d[1], dHz = d[2], dEx = d[3], dEy = d[4], dEz = d[5];
    const R ndH = nx * dHx + ny * dHy + nz * dHz;
    const R ndE = nx * dEx + ny * dEy + nz * dEz;
    const R cEx = ny * dEz - nz * dEy, cEy = nz * dEx - nx * dEz, cEz = nx * dEy - ny * dEx;
    const R cHx = ny * dHz - nz * dHy, cHy = nz * dHx - nx * dHz, cHz = nx * dHy - ny * dHx;
    fl[0] = h * cEx + ah * (nx * ndH - dHx);
    fl[1] = h * cEy + ah * (ny * ndH - dHy);
    fl[2] = h * cEz + ah * (nz * ndH - dHz);
    fl[3] = -h * cHx + ah * (nx * ndE - dEx);
    fl[4] = -h * cHy + ah * (ny * ndE - dEy);
    fl[5] = -h * cHz + ah * (nz * ndE - dEz);
}

}  // namespace

// Face nodes of partner traces kept in flight ahead of their use (FP32: one
// face node per K step; split: eight per K step).
#ifndef DGW_3D_SPD
#define DGW_3D_SPD 2
#endif
#ifndef DGW_3D_SPD_SPLIT
#define DGW_3D_SPD_SPLIT 2
#endif
// FP32: the next work unit's factors and first operands loaded before this
// unit's update (1) or at the next unit's start (0).
#ifndef DGW_3D_NPF
#define DGW_3D_NPF 0
#endif
// Fields whose residual runs are loaded before the surface loop (the rest at
// the update).
#ifndef DGW_3D_RPF
#define DGW_3D_RPF 6
#endif
#ifndef DGW_3D_RPF_SPLIT
#define DGW_3D_RPF_SPLIT 0
#endif
// Surface-loop K step at which the other fields' residual runs are loaded
// (negative: at the update).
#ifndef DGW_3D_RAT
#define DGW_3D_RAT -1
#endif
#ifndef DGW_3D_RAT_SPLIT
#define DGW_3D_RAT_SPLIT -1
#endif
// Scheduling fences of the FP32 kernel: bit 0 after each volume field, bit 1
// after each LIFT K step (they bound the registers the compiler keeps live).
#ifndef DGW_3D_SB
#define DGW_3D_SB 3
#endif
// Fields of FP32 volume operands in flight ahead of their contraction.
#ifndef DGW_3D_VPD
#define DGW_3D_VPD 1
#endif

// SHARE: partner traces inside the work-group's pair of tiles come from the
// other waves' LDS copies (the work partition the library runs by default);
// without it a wave reads only its own LDS copy and the tile loop has no
// work-group barriers (a candidate of the automated tuning).
template <int N, bool SPLIT, bool SHARE>
__global__ void __launch_bounds__(512) stage3d_kernel(StageArgs A) {
    using T = Tet<N>;
    constexpr int Np = T::Np, Nfp = T::Nfp, Nafp = T::Nafp, NPP = T::NPP, KV = T::KV, NC = T::NC, NR = T::NR;
    constexpr int MTD = T::MTD, MTL = T::MTL, KL = T::KL, KVS = T::KVS, KLS = T::KLS, RS = T::RS, ES = T::ES;
    constexpr int AV = T::AV, AL = T::AL, FV = T::FV, FL = T::FL, FT = T::FT, KT = T::KT, NT = T::NT;
    constexpr int FRAG4 = SPLIT ? 2 * FV + FL + (FT + 3) / 4 : (AV + AL + 3) / 4;  // in 16-byte units
    __shared__ uint4 sAq[FRAG4];
    __shared__ int stab[NT];
    // split: each wave's FP64 face data of its 16 elements, [element][face * 4 + q]
    // (n_x, n_y, n_z, Fscale), read per face node; an element stride of 17
    // doubles puts the 16 elements of a lane group in different banks
    __shared__ double sfd[SPLIT ? 8 : 1][16][17];
    // each wave's copy of its 16 elements' fields, [element][field][node],
    // element stride ES
    __shared__ __attribute__((aligned(16))) float sF[8][16 * ES];
    const float *sA = reinterpret_cast<const float *>(sAq);

    {
        const uint4 *src = reinterpret_cast<const uint4 *>(A.opsfrag);
        for (int i = threadIdx.x; i < FRAG4; i += 512) sAq[i] = src[i];
        for (int i = threadIdx.x; i < NT; i += 512) stab[i] = A.itab[i];
    }
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

    float *F = sF[w];
    // FP32 with DGW_3D_NPF: the next work unit's factors and first field's
    // operands, loaded during this unit's surface phase
    float nG[9], nb0[Tet<N>::KV];
    bool npf_ok = false;
    // gathered partner traces of the face-node slots in flight: zeroed once
    // here, not per unit (a per-unit zero of the in-window lanes after the
    // masked loads of the others would make the compiler wait for those
    // loads right away, before the barrier they are meant to cross)
    float rval[SPLIT ? DGW_3D_SPD_SPLIT : DGW_3D_SPD][6];
#pragma unroll
    for (int t = 0; t < (SPLIT ? DGW_3D_SPD_SPLIT : DGW_3D_SPD); ++t)
#pragma unroll
        for (int f = 0; f < 6; ++f) rval[t][f] = 0.f;
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
        constexpr unsigned TB = 64 * RS * 4;  // bytes of a tile's fields
        const __amdgpu_buffer_rsrc_t rq = rsrc(A.qin + (size_t)tile * (64 * RS), TB);
        const unsigned vel = (unsigned)(col * RS) * 4;   // the lane's element
        const unsigned v16 = vel + 16u * (unsigned)g;    // its first 16-byte run
        const unsigned v4 = vel + 4u * (unsigned)g;      // its first single node
        float *Fc = F + c * ES;
        const unsigned vcol = (unsigned)col * 4;         // column of a tiled factor row

        float cv[6][KV];  // volume part of the right-hand side, nodes of the lane
#pragma unroll
        for (int o = 0; o < 6; ++o)
#pragma unroll
            for (int i = 0; i < KV; ++i) cv[o][i] = 0.f;

        if (active) {
            if constexpr (!SPLIT) {
                // ---- FP32 volume: operands of field f are the lane's nodes
                // (K row 4 ks + g = node slot ks); the next field's are in
                // flight while field f is contracted
                float G[9];
                if (DGW_3D_NPF && npf_ok) {
#pragma unroll
                    for (int q = 0; q < 9; ++q) G[q] = nG[q];
                } else {
                    const __amdgpu_buffer_rsrc_t rg = rsrc(A.geo + (size_t)tile * (9 * 64), 9 * 64 * 4);
#pragma unroll
                    for (int q = 0; q < 9; ++q) G[q] = bload(rg, vcol, q * 256);
                }
                auto load_b = [&](int f, float (&b)[KV]) {
#pragma unroll
                    for (int t = 0; t < NC; ++t) bload4(rq, v16, (f * NPP + 16 * t) * 4, &b[4 * t]);
#pragma unroll
                    for (int r = 0; r < NR; ++r) b[4 * NC + r] = bload(rq, v4, (f * NPP + 16 * NC + 4 * r) * 4);
                };
                // operands of the next VPD fields in flight (a ring)
                constexpr int VPD = DGW_3D_VPD;
                float bn[VPD][KV];
#pragma unroll
                for (int f0 = 0; f0 < VPD; ++f0) {
                    if (f0 == 0 && DGW_3D_NPF && npf_ok) {
#pragma unroll
                        for (int i = 0; i < KV; ++i) bn[0][i] = nb0[i];
                    } else {
                        load_b(f0, bn[f0]);
                    }
                }
                auto field = [&](auto FI) {
                    constexpr int f = decltype(FI)::value;
                    float b[KV];
#pragma unroll
                    for (int i = 0; i < KV; ++i) b[i] = bn[f % VPD][i];
                    // the wave's LDS copy of field f
#pragma unroll
                    for (int t = 0; t < NC; ++t)
                        *reinterpret_cast<floatx4 *>(Fc + f * NPP + 16 * t + 4 * g) =
                            floatx4{b[4 * t], b[4 * t + 1], b[4 * t + 2], b[4 * t + 3]};
#pragma unroll
                    for (int r = 0; r < NR; ++r) Fc[f * NPP + 16 * NC + 4 * r + g] = b[4 * NC + r];
                    if constexpr (f + VPD < 6) load_b(f + VPD, bn[f % VPD]);
                    floatx4 d[MTD];
#pragma unroll
                    for (int m = 0; m < MTD; ++m) d[m] = floatx4{0.f, 0.f, 0.f, 0.f};
                    // operator fragments re-read from LDS for every field (an
                    // index opaque to the compiler keeps them out of registers)
                    int la = lane;
                    asm volatile("" : "+v"(la));
#pragma unroll
                    for (int ks = 0; ks < KV; ++ks)
#pragma unroll
                        for (int m = 0; m < MTD; ++m)
                            d[m] = __builtin_amdgcn_mfma_f32_16x16x4f32(sA[(m * KV + ks) * 64 + la], b[ks], d[m], 0, 0, 0);
                    // chain rule: slot 3 i + p holds D_p of node slot i
#pragma unroll
                    for (int i = 0; i < KV; ++i) {
                        const float dr = d[(3 * i) / 4][(3 * i) % 4], ds = d[(3 * i + 1) / 4][(3 * i + 1) % 4];
                        const float dtt = d[(3 * i + 2) / 4][(3 * i + 2) % 4];
                        const float gx = G[0] * dr + G[3] * ds + G[6] * dtt;
                        const float gy = G[1] * dr + G[4] * ds + G[7] * dtt;
                        const float gz = G[2] * dr + G[5] * ds + G[8] * dtt;
                        curl_add<f>(gx, gy, gz, cv[0][i], cv[1][i], cv[2][i], cv[3][i], cv[4][i], cv[5][i]);
                    }
                    // materialise the sums here: otherwise they are sunk to
                    // their use and every field's derivatives stay live
#pragma unroll
                    for (int o = 0; o < 6; ++o)
#pragma unroll
                        for (int i = 0; i < KV; ++i) asm volatile("" : "+v"(cv[o][i]));
                    if (DGW_3D_SB & 1) __builtin_amdgcn_sched_barrier(0);
                };
                field(std::integral_constant<int, 0>{});
                field(std::integral_constant<int, 1>{});
                field(std::integral_constant<int, 2>{});
                field(std::integral_constant<int, 3>{});
                field(std::integral_constant<int, 4>{});
                field(std::integral_constant<int, 5>{});
            } else {
                // ---- split volume: K step ks, lane group g holds the nodes
                // 32 ks + 8 g .. + 7 (two 16-byte runs; runs past the field
                // meet zero operator columns and are not loaded)
                double G[9];
                {
                    const double *gt = A.geo64 + (size_t)tile * (9 * 64);
#pragma unroll
                    for (int q = 0; q < 9; ++q) G[q] = gt[(unsigned)(q * 64 + col)];
                }
                const unsigned v8 = vel + 32u * (unsigned)g;
                constexpr int KTA = KT > 0 ? KT : 1;
                // 16-bit K steps (b), then the FP32 tail: K row 4 kt + g of
                // the tail is node 32 KVS + 4 kt + g (bt)
                auto load_b = [&](int f, float (&b)[KVS][8], float (&bt)[KTA]) {
#pragma unroll
                    for (int ks = 0; ks < KVS; ++ks)
#pragma unroll
                        for (int h = 0; h < 2; ++h) {
                            if (32 * ks + 8 * g + 4 * h < NPP)
                                bload4(rq, v8, (f * NPP + 32 * ks + 4 * h) * 4, &b[ks][4 * h]);
                            else
#pragma unroll
                                for (int k = 0; k < 4; ++k) b[ks][4 * h + k] = 0.f;
                        }
#pragma unroll
                    for (int kt = 0; kt < KT; ++kt) bt[kt] = bload(rq, v4, (f * NPP + 32 * KVS + 4 * kt) * 4);
                };
                float bn[KVS][8], btn[KTA];
                float qcn = bload(rq, vel, 0);
                load_b(0, bn, btn);
                auto field = [&](auto FI) {
                    constexpr int f = decltype(FI)::value;
                    float b[KVS][8], bt[KTA];
                    const float qc = qcn;
#pragma unroll
                    for (int ks = 0; ks < KVS; ++ks)
#pragma unroll
                        for (int q = 0; q < 8; ++q) b[ks][q] = bn[ks][q];
#pragma unroll
                    for (int kt = 0; kt < KTA; ++kt) bt[kt] = btn[kt];
#pragma unroll
                    for (int ks = 0; ks < KVS; ++ks)
#pragma unroll
                        for (int h = 0; h < 2; ++h)
                            if (32 * ks + 8 * g + 4 * h < NPP)
                                *reinterpret_cast<floatx4 *>(Fc + f * NPP + 32 * ks + 8 * g + 4 * h) =
                                    floatx4{b[ks][4 * h], b[ks][4 * h + 1], b[ks][4 * h + 2], b[ks][4 * h + 3]};
#pragma unroll
                    for (int kt = 0; kt < KT; ++kt) Fc[f * NPP + 32 * KVS + 4 * kt + g] = bt[kt];
                    if constexpr (f + 1 < 6) {
                        qcn = bload(rq, vel, (f + 1) * NPP * 4);
                        load_b(f + 1, bn, btn);
                    }
                    floatx4 d[MTD];
#pragma unroll
                    for (int m = 0; m < MTD; ++m) d[m] = floatx4{0.f, 0.f, 0.f, 0.f};
                    int la = lane;
                    asm volatile("" : "+v"(la));
#pragma unroll
                    for (int ks = 0; ks < KVS; ++ks) {
                        bf16x8 bh, bl;
#pragma unroll
                        for (int q = 0; q < 8; ++q) {
                            const float v = b[ks][q] - qc;
                            const __bf16 hh = (__bf16)v;
                            bh[q] = hh;
                            bl[q] = (__bf16)(v - (float)hh);
                        }
#pragma unroll
                        for (int m = 0; m < MTD; ++m) {
                            const int fi = (m * KVS + ks) * 64 + la;
                            d[m] = mfma3(as_bf16x8(sAq[fi]), as_bf16x8(sAq[FV + fi]), bh, bl, d[m]);
                        }
                    }
                    const float *sT = reinterpret_cast<const float *>(sAq + 2 * FV + FL);
#pragma unroll
                    for (int kt = 0; kt < KT; ++kt)
#pragma unroll
                        for (int m = 0; m < MTD; ++m)
                            d[m] = __builtin_amdgcn_mfma_f32_16x16x4f32(sT[(m * KT + kt) * 64 + la], bt[kt] - qc, d[m], 0, 0,
                                                                        0);
                    // chain rule and curl in FP64 with the FP64 factors
#pragma unroll
                    for (int i = 0; i < KV; ++i) {
                        const double dr = d[(3 * i) / 4][(3 * i) % 4], ds = d[(3 * i + 1) / 4][(3 * i + 1) % 4];
                        const double dtt = d[(3 * i + 2) / 4][(3 * i + 2) % 4];
                        const double gx = G[0] * dr + G[3] * ds + G[6] * dtt;
                        const double gy = G[1] * dr + G[4] * ds + G[7] * dtt;
                        const double gz = G[2] * dr + G[5] * ds + G[8] * dtt;
                        curl_add<f>(gx, gy, gz, cv[0][i], cv[1][i], cv[2][i], cv[3][i], cv[4][i], cv[5][i]);
                    }
#pragma unroll
                    for (int o = 0; o < 6; ++o)
#pragma unroll
                        for (int i = 0; i < KV; ++i) asm volatile("" : "+v"(cv[o][i]));
                    __builtin_amdgcn_sched_barrier(0);
                };
                field(std::integral_constant<int, 0>{});
                field(std::integral_constant<int, 1>{});
                field(std::integral_constant<int, 2>{});
                field(std::integral_constant<int, 3>{});
                field(std::integral_constant<int, 4>{});
                field(std::integral_constant<int, 5>{});
            }
        }  // active

        // ---- surface.  Face records of the element, held as scalars
        // (selected per lane, no per-lane array indexing)
        int rc0 = -1, rc1 = -1, rc2 = -1, rc3 = -1;
        if (active) {
            const __amdgpu_buffer_rsrc_t rn = rsrc(A.nbr + (size_t)tile * (4 * 64), 4 * 64 * 4);
            rc0 = __builtin_bit_cast(int, bload(rn, vcol, 0));
            rc1 = __builtin_bit_cast(int, bload(rn, vcol, 256));
            rc2 = __builtin_bit_cast(int, bload(rn, vcol, 512));
            rc3 = __builtin_bit_cast(int, bload(rn, vcol, 768));
        }
        auto face_rec = [&](int face) { return face == 0 ? rc0 : face == 1 ? rc1 : face == 2 ? rc2 : rc3; };
        // all partner traces outside the pair through one resource over the
        // field array
        const __amdgpu_buffer_rsrc_t rall = rsrc(A.qin, (unsigned)A.ntiles * TB);
        // where the partner trace of face node j lives: element e2, node pn;
        // on the wall the element itself (the mirror sign is applied with the
        // jump); inpair: e2 lies in this pair of tiles (LDS copy)
        struct Partner {
            int own, e2, pn;
            bool wall, inpair;
        };
        auto partner = [&](int j) {
            Partner P;
            const int jc = j < Nafp ? j : Nafp - 1;  // padding rows read a valid node
            const int face = jc / Nfp, i = jc - face * Nfp;
            P.own = stab[jc];
            const int rc = face_rec(face);
            P.wall = rc < 0;
            P.e2 = P.wall ? tile * 64 + col : (rc >> 5);
            P.pn = P.wall ? P.own : stab[Nafp + (((rc >> 3) & 3) * 6 + (rc & 7)) * Nfp + i];
            // without SHARE only the wave's own 16 elements count
            P.inpair = SHARE ? (unsigned)((P.e2 >> 6) - 2 * pair) < 2u : (P.e2 >> 4) == ((tile * 64 + col) >> 4);
            return P;
        };
        // face node of this lane at slot t: FP32 one per K step (4 ks + g),
        // split four per K step (16 ks + 4 g + q)
        constexpr int NS = SPLIT ? 4 * KLS : KL;
        constexpr int SPD = SPLIT ? DGW_3D_SPD_SPLIT : DGW_3D_SPD;
        auto slot_j = [&](int t) { return SPLIT ? 16 * (t / 4) + 4 * g + t % 4 : 4 * t + g; };
        // Where the traces of slot t live is worked out once, SPD slots ahead
        // of their use (the first ones across the barrier below): the own
        // node and the wall flag (rown), the partner's LDS offset when it lies
        // in the pair (rloc >= 0), else its six values gathered from memory
        // (rval)
        int rown[SPD], rloc[SPD];
        const float *sFf = &sF[0][0];
        auto gather = [&](int t, int slot) {
            const Partner P = partner(slot_j(t));
            rown[slot] = P.own | (P.wall ? 256 : 0);
            if (P.inpair) {
                const int t2 = (P.e2 >> 6) - 2 * pair;
                rloc[slot] = ((4 * t2 + ((P.e2 & 63) >> 4)) * 16 + (P.e2 & 15)) * ES + P.pn;
            } else {
                rloc[slot] = -1;
                const unsigned vp = ((unsigned)P.e2 * RS + P.pn) * 4;
#pragma unroll
                for (int f = 0; f < 6; ++f) rval[slot][f] = bload(rall, vp, f * NPP * 4);
            }
        };
        // own and partner traces of the slot's face node; returns the wall flag
        auto traces = [&](int t, int slot, float (&m)[6], float (&pv)[6]) {
            (void)t;
            const int own = rown[slot] & 255, loc = rloc[slot];
#pragma unroll
            for (int f = 0; f < 6; ++f) m[f] = Fc[f * NPP + own];
            if (loc >= 0) {
#pragma unroll
                for (int f = 0; f < 6; ++f) pv[f] = sFf[loc + f * NPP];
            } else {
#pragma unroll
                for (int f = 0; f < 6; ++f) pv[f] = rval[slot][f];
            }
            return (rown[slot] & 256) != 0;
        };
#pragma unroll
        for (int t = 0; t < SPD; ++t) {
            rown[t] = 0;
            rloc[t] = 0;
        }
        if (active) {
#pragma unroll
            for (int t = 0; t < SPD; ++t)
                if (t < NS) gather(t, t);
        }
        // every wave's LDS copy of its fields is complete: partner traces of
        // elements in this pair of tiles are read from there
        if (SHARE) __syncthreads();
        if (active) {
            // residual runs of the first RPF fields: loaded here, used in the
            // update after the surface loop (their latency hides behind it)
            const __amdgpu_buffer_rsrc_t rr = rsrc(A.res + (size_t)tile * (64 * RS), TB);
            const __amdgpu_buffer_rsrc_t ro = rsrc(A.qout + (size_t)tile * (64 * RS), TB);
            constexpr int RPF = SPLIT ? DGW_3D_RPF_SPLIT : DGW_3D_RPF;
            // K step of the surface loop at which the remaining residual runs
            // are loaded (negative: at the update)
            constexpr int RAT = SPLIT ? DGW_3D_RAT_SPLIT : DGW_3D_RAT;
            float rv[6][KV];
            auto load_res = [&](int f) {
#pragma unroll
                for (int t = 0; t < NC; ++t) bload4(rr, v16, (f * NPP + 16 * t) * 4, &rv[f][4 * t]);
#pragma unroll
                for (int r = 0; r < NR; ++r) rv[f][4 * NC + r] = bload(rr, v4, (f * NPP + 16 * NC + 4 * r) * 4);
            };
#pragma unroll
            for (int f = 0; f < RPF; ++f) load_res(f);
            if (RPF > 0) __builtin_amdgcn_sched_barrier(0);  // issued here, not sunk to the update
            // the LIFT contraction accumulates on top of the volume part:
            // slot 4 mt + jj of lane group g = node slot i
            floatx4 acc[6][MTL];
#pragma unroll
            for (int o = 0; o < 6; ++o)
#pragma unroll
                for (int mt = 0; mt < MTL; ++mt)
#pragma unroll
                    for (int jj = 0; jj < 4; ++jj) {
                        constexpr int dummy = 0;
                        const int i = 4 * mt + jj;
                        acc[o][mt][jj] = i < KV ? cv[o][i < KV ? i : dummy] : 0.f;
                    }

            if constexpr (!SPLIT) {
                float fd[16];
                {
                    const __amdgpu_buffer_rsrc_t rf = rsrc(A.fgeo + (size_t)tile * (16 * 64), 16 * 64 * 4);
#pragma unroll
                    for (int q = 0; q < 16; ++q) fd[q] = bload(rf, vcol, q * 256);
                }
                const float ha = 0.5f * A.alpha;
                // FP32 LIFT, K step ks: lane group g evaluates face node 4 ks + g
#pragma unroll
                for (int ks = 0; ks < KL; ++ks) {
                    if (ks == RAT) {
#pragma unroll
                        for (int f = RPF; f < 6; ++f) load_res(f);
                    }
                    const int j = 4 * ks + g;
                    float m[6], pv[6];
                    const bool wall = traces(ks, ks % SPD, m, pv);
                    if (ks + SPD < KL) gather(ks + SPD, ks % SPD);
                    // the four face nodes of a K step lie on at most two faces,
                    // lo and hi (fixed once the loop is unrolled): a two-way
                    // select with constant indices
                    constexpr int dummy = 0;
                    const int flo = (4 * ks < Nafp ? 4 * ks : Nafp - 1) / Nfp;
                    const int fhi = flo + 1 < 4 ? flo + 1 : 3;
                    const bool hi = (j < Nafp ? j : Nafp - 1) >= Nfp * (flo + 1);
                    auto fv = [&](int q) { return hi ? fd[4 * fhi + q + dummy] : fd[4 * flo + q + dummy]; };
                    float dq[6];
#pragma unroll
                    for (int f = 0; f < 6; ++f) dq[f] = m[f] - ((wall && f >= 3) ? -pv[f] : pv[f]);
                    const float fs = fv(3);
                    const float h = j < Nafp ? 0.5f * fs : 0.f, ah = j < Nafp ? ha * fs : 0.f;
                    float fl[6];
                    face_flux<float>(dq, fv(0), fv(1), fv(2), h, ah, fl);
#pragma unroll
                    for (int mt = 0; mt < MTL; ++mt) {
                        const float a = sA[AV + (mt * KL + ks) * 64 + lane];
#pragma unroll
                        for (int f = 0; f < 6; ++f)
                            acc[f][mt] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, fl[f], acc[f][mt], 0, 0, 0);
                    }
                    if (DGW_3D_SB & 2) __builtin_amdgcn_sched_barrier(0);
                }
            } else {
                {
                    // lane group g fetches face g of its element
                    const double *ft = A.fgeo64 + (size_t)tile * (16 * 64);
#pragma unroll
                    for (int q = 0; q < 4; ++q) sfd[w][c][4 * g + q] = ft[(unsigned)((4 * g + q) * 64 + col)];
                }
                auto face_val = [&](int face, int q) { return sfd[w][c][4 * face + q]; };
                const double ha = 0.5 * (double)A.alpha;
                // split LIFT, K step ks (16 face-node rows): lane group g
                // evaluates face nodes 16 ks + 4 g + q, q = 0..3
                const uint2 *sL = reinterpret_cast<const uint2 *>(sAq + 2 * FV);
#pragma unroll
                for (int ks = 0; ks < KLS; ++ks) {
                    if (ks == RAT) {
#pragma unroll
                        for (int f = RPF; f < 6; ++f) load_res(f);
                    }
                    // hi and lo parts of the flux rows, two BF16 per word
                    unsigned bhw[6][2], blw[6][2];
#pragma unroll
                    for (int q2 = 0; q2 < 2; ++q2) {
                        float fl2[2][6];
#pragma unroll
                        for (int u = 0; u < 2; ++u) {
                            const int t = 4 * ks + 2 * q2 + u;
                            const int j = 16 * ks + 4 * g + 2 * q2 + u;
                            float m[6], pv[6];
                            const bool wall = traces(t, t % SPD, m, pv);
                            if (t + SPD < NS) gather(t + SPD, t % SPD);
                            const int face = (j < Nafp ? j : Nafp - 1) / Nfp;
                            double dq[6];
#pragma unroll
                            for (int f = 0; f < 6; ++f)
                                dq[f] = (double)m[f] - ((wall && f >= 3) ? -(double)pv[f] : (double)pv[f]);
                            const double fs = face_val(face, 3);
                            const double h = j < Nafp ? 0.5 * fs : 0.0, ah = j < Nafp ? ha * fs : 0.0;
                            double fl[6];
                            face_flux<double>(dq, face_val(face, 0), face_val(face, 1), face_val(face, 2), h, ah, fl);
#pragma unroll
                            for (int f = 0; f < 6; ++f) fl2[u][f] = (float)fl[f];
                        }
#pragma unroll
                        for (int f = 0; f < 6; ++f) {
                            const bf16x2 hh = __builtin_convertvector((float2v){fl2[0][f], fl2[1][f]}, bf16x2);
                            const bf16x2 ll = __builtin_convertvector(
                                (float2v){fl2[0][f] - (float)hh[0], fl2[1][f] - (float)hh[1]}, bf16x2);
                            bhw[f][q2] = __builtin_bit_cast(unsigned, hh);
                            blw[f][q2] = __builtin_bit_cast(unsigned, ll);
                        }
                        __builtin_amdgcn_sched_barrier(0);
                    }
#pragma unroll
                    for (int mt = 0; mt < MTL; ++mt) {
                        const int fi = (mt * KLS + ks) * 64 + lane;
                        const shortx4 ah16 = __builtin_bit_cast(shortx4, sL[fi]), al16 = __builtin_bit_cast(shortx4, sL[FL + fi]);
#pragma unroll
                        for (int f = 0; f < 6; ++f) {
                            const shortx4 bh = __builtin_bit_cast(shortx4, uint2{bhw[f][0], bhw[f][1]});
                            const shortx4 bl = __builtin_bit_cast(shortx4, uint2{blw[f][0], blw[f][1]});
                            floatx4 c = acc[f][mt];
                            c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah16, bh, c, 0, 0, 0);
                            c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah16, bl, c, 0, 0, 0);
                            acc[f][mt] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(al16, bh, c, 0, 0, 0);
                        }
                    }
                    __builtin_amdgcn_sched_barrier(0);
                }
            }

            // the next unit's factors and first operands (FP32, DGW_3D_NPF)
            if constexpr (!SPLIT && DGW_3D_NPF) {
                const int pl2 = pl + GB, tile2 = 2 * (xbase + pl2) + (w >> 2);
                npf_ok = pl2 < xcount && tile2 < A.ntiles;  // wave-uniform
                if (npf_ok) {
                    const __amdgpu_buffer_rsrc_t rg2 = rsrc(A.geo + (size_t)tile2 * (9 * 64), 9 * 64 * 4);
#pragma unroll
                    for (int q = 0; q < 9; ++q) nG[q] = bload(rg2, vcol, q * 256);
                    const __amdgpu_buffer_rsrc_t rq2 = rsrc(A.qin + (size_t)tile2 * (64 * RS), TB);
#pragma unroll
                    for (int t = 0; t < NC; ++t) bload4(rq2, v16, (16 * t) * 4, &nb0[4 * t]);
#pragma unroll
                    for (int r = 0; r < NR; ++r) nb0[4 * NC + r] = bload(rq2, v4, (16 * NC + 4 * r) * 4);
                }
            }
            // ---- fused low-storage RK update of the lane's nodes: every
            // residual load first (their latencies overlap; the first RPF
            // fields' were issued before the surface loop), then per field
            // the arithmetic and the stores
#pragma unroll
            for (int f = RPF; f < 6; ++f)
                if (RAT < 0 || RAT >= (SPLIT ? KLS : KL)) load_res(f);
#pragma unroll
            for (int f = 0; f < 6; ++f) {
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
                    if (16 * NC + 4 * r + g < Np) {  // pad nodes stay 0
                        bstore(rr, rv[f][4 * NC + r], v4, (f * NPP + 16 * NC + 4 * r) * 4);
                        bstore(ro, qv[4 * NC + r], v4, (f * NPP + 16 * NC + 4 * r) * 4);
                    }
            }
        }  // active
        if (SHARE) __syncthreads();  // the LDS copies are read by other waves until here
    }
}

template <int N, bool SPLIT, bool SHARE>
static hipError_t launch3d(const StageArgs &a, hipStream_t s) {
    // every pointer the kernel dereferences must be set
    if (!a.opsfrag || !a.itab || !a.qin || !a.qout || !a.res || !a.nbr || a.ntiles <= 0 || a.ngroups < 8 ||
        (a.ngroups & 7))
        return hipErrorInvalidValue;
    if (SPLIT ? (!a.geo64 || !a.fgeo64) : (!a.geo || !a.fgeo)) return hipErrorInvalidValue;
    hipLaunchKernelGGL((stage3d_kernel<N, SPLIT, SHARE>), dim3(a.ngroups), dim3(512), 0, s, a);
    return hipGetLastError();
}

template <int N, bool SPLIT, bool SHARE>
static int occupancy3d() {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, stage3d_kernel<N, SPLIT, SHARE>, 512, 0) != hipSuccess)
        return 1;
    return nb > 0 ? nb : 1;
}

template <bool SPLIT, bool SHARE>
static hipError_t launch3d_n(int N, const StageArgs &a, hipStream_t s) {
    switch (N) {
        case 1: return launch3d<1, SPLIT, SHARE>(a, s);
        case 2: return launch3d<2, SPLIT, SHARE>(a, s);
        case 3: return launch3d<3, SPLIT, SHARE>(a, s);
        case 4: return launch3d<4, SPLIT, SHARE>(a, s);
        default: return hipErrorInvalidValue;
    }
}

template <bool SPLIT, bool SHARE>
static int occupancy3d_n(int N) {
    switch (N) {
        case 1: return occupancy3d<1, SPLIT, SHARE>();
        case 2: return occupancy3d<2, SPLIT, SHARE>();
        case 3: return occupancy3d<3, SPLIT, SHARE>();
        case 4: return occupancy3d<4, SPLIT, SHARE>();
        default: return 1;
    }
}

int blocks_per_cu_3d(int N, bool share) { return share ? occupancy3d_n<false, true>(N) : occupancy3d_n<false, false>(N); }
int blocks_per_cu_3d_split(int N, bool share) {
    return share ? occupancy3d_n<true, true>(N) : occupancy3d_n<true, false>(N);
}
hipError_t launch_stage3d(int N, bool share, const StageArgs &a, hipStream_t s) {
    return share ? launch3d_n<false, true>(N, a, s) : launch3d_n<false, false>(N, a, s);
}
hipError_t launch_stage3d_split(int N, bool share, const StageArgs &a, hipStream_t s) {
    return share ? launch3d_n<true, true>(N, a, s) : launch3d_n<true, false>(N, a, s);
}

const char *stage3d_kernel_name(int N) {
    (void)N;
    return "stage3d_kernel<N, false, true>";
}

namespace {

// Output slot of row r (0..15) of M-tile mt: lane group r / 4, slot
// 4 mt + r % 4.
struct OutSlot {
    int g, s;
};
inline OutSlot out_slot(int mt, int r) { return {r / 4, 4 * mt + r % 4}; }

uint16_t bf16_bits(float f) {
    uint32_t u;
    __builtin_memcpy(&u, &f, 4);
    return (uint16_t)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);  // nearest even (finite inputs)
}
float bf16_value(uint16_t h) {
    const uint32_t u = (uint32_t)h << 16;
    float f;
    __builtin_memcpy(&f, &u, 4);
    return f;
}

// Entry of the packed derivative operator at output slot (g, s) and node
// column n (0 outside): D_(s mod 3)[node of slot s / 3][n].
double deriv_entry(int N, const double *const D[3], int g, int s, int n) {
    const int Np = (N + 1) * (N + 2) * (N + 3) / 6, KV = npp_pad(Np) / 4;
    if (s >= 3 * KV) return 0.0;
    const int no = slot_node(KV, g, s / 3);
    return (no < Np && n >= 0 && n < Np) ? D[s % 3][(size_t)no * Np + n] : 0.0;
}
// Entry of the row-permuted LIFT at output slot (g, s) and face node j.
double lift_entry(int N, const double *LIFT, int g, int s, int j) {
    const int Np = (N + 1) * (N + 2) * (N + 3) / 6, KV = npp_pad(Np) / 4, Nafp = 2 * (N + 1) * (N + 2);
    if (s >= KV) return 0.0;
    const int no = slot_node(KV, g, s);
    return (no < Np && j < Nafp) ? LIFT[(size_t)no * Nafp + j] : 0.0;
}

}  // namespace

// A-fragment order of the FP32 3D kernel's operators: the packed derivative
// operator, out[(mt*KV + ks)*64 + l] = row (mt, l % 16), K row 4 ks + l / 16
// (= node slot_node(KV, l / 16 % 4, ks)), then LIFT,
// out[AV + (mt*KL + ks)*64 + l] = row (mt, l % 16), face node 4 ks + l / 16.
// Returns the number of floats.
int opsfrag3d(int N, const double *Dr, const double *Ds, const double *Dt, const double *LIFT, float *out) {
    const int Np = (N + 1) * (N + 2) * (N + 3) / 6, Nafp = 2 * (N + 1) * (N + 2);
    const int KV = npp_pad(Np) / 4, MTD = (3 * KV + 3) / 4, MTL = (KV + 3) / 4, KL = (Nafp + 3) / 4;
    const int AV = MTD * KV * 64, AL = MTL * KL * 64;
    if (!out) return AV + AL;
    const double *D[3] = {Dr, Ds, Dt};
    for (int mt = 0; mt < MTD; ++mt)
        for (int ks = 0; ks < KV; ++ks)
            for (int l = 0; l < 64; ++l) {
                const OutSlot o = out_slot(mt, l % 16);
                const int kg = l / 16;  // K row 4 ks + kg: node of slot ks of lane group kg
                out[(mt * KV + ks) * 64 + l] = (float)deriv_entry(N, D, o.g, o.s, slot_node(KV, kg, ks));
            }
    for (int mt = 0; mt < MTL; ++mt)
        for (int ks = 0; ks < KL; ++ks)
            for (int l = 0; l < 64; ++l) {
                const OutSlot o = out_slot(mt, l % 16);
                out[AV + (mt * KL + ks) * 64 + l] = (float)lift_entry(N, LIFT, o.g, o.s, 4 * ks + l / 16);
            }
    return AV + AL;
}

// Split operator fragments of the split 3D kernel: the derivative blocks
// (mt, ks) x 64 lanes x 8 BF16, hi part then lo part (lane l holds row
// (mt, l % 16) at node columns 32 ks + 8 (l / 16) + q, q = 0..7); the LIFT
// blocks (mt, ks) x 64 lanes x 4 BF16, hi then lo (face nodes
// 16 ks + 4 (l / 16) + q, q = 0..3); the FP32 tail of the derivative.
// Returns the size in bytes (out == nullptr: size only).
int opsfrag3d_split(int N, const double *Dr, const double *Ds, const double *Dt, const double *LIFT, void *out) {
    const int Np = (N + 1) * (N + 2) * (N + 3) / 6, Nafp = 2 * (N + 1) * (N + 2), NPP = npp_pad(Np);
    const int KV = NPP / 4, MTD = (3 * KV + 3) / 4, MTL = (KV + 3) / 4;
    const int TAILN = NPP % 32;
    const bool tail = NPP >= 32 && TAILN > 0 && TAILN <= 8;
    const int KVS = tail ? NPP / 32 : (NPP + 31) / 32, KT = tail ? TAILN / 4 : 0, KLS = (Nafp + 15) / 16;
    const int FV = MTD * KVS * 64, FL = MTL * KLS * 64, FT = MTD * KT * 64;
    const size_t total = (size_t)2 * FV * 16 + (size_t)2 * FL * 8 + (size_t)FT * 4;
    if (!out) return (int)total;
    // 16-bit words: derivative hi [0, 8 FV), lo [8 FV, 16 FV); LIFT hi
    // [16 FV, 16 FV + 4 FL), lo after it; then the FP32 tail
    uint16_t *o16 = static_cast<uint16_t *>(out);
    auto split16 = [](double v, uint16_t &hi, uint16_t &lo) {
        hi = bf16_bits((float)v);
        lo = bf16_bits((float)(v - (double)bf16_value(hi)));
    };
    const double *D[3] = {Dr, Ds, Dt};
    for (int mt = 0; mt < MTD; ++mt)
        for (int ks = 0; ks < KVS; ++ks)
            for (int l = 0; l < 64; ++l) {
                const OutSlot o = out_slot(mt, l % 16);
                const size_t frag = (size_t)(mt * KVS + ks) * 64 + l;
                for (int q = 0; q < 8; ++q)
                    split16(deriv_entry(N, D, o.g, o.s, 32 * ks + 8 * (l / 16) + q), o16[frag * 8 + q],
                            o16[(size_t)FV * 8 + frag * 8 + q]);
            }
    const size_t lift0 = (size_t)16 * FV;
    for (int mt = 0; mt < MTL; ++mt)
        for (int ks = 0; ks < KLS; ++ks)
            for (int l = 0; l < 64; ++l) {
                const OutSlot o = out_slot(mt, l % 16);
                const size_t frag = (size_t)(mt * KLS + ks) * 64 + l;
                for (int q = 0; q < 4; ++q)
                    split16(lift_entry(N, LIFT, o.g, o.s, 16 * ks + 4 * (l / 16) + q), o16[lift0 + frag * 4 + q],
                            o16[lift0 + (size_t)FL * 4 + frag * 4 + q]);
            }
    // FP32 tail of the derivative: row (mt, l % 16), K row 4 kt + l / 16 =
    // node 32 KVS + 4 kt + l / 16
    float *t32 = reinterpret_cast<float *>(static_cast<char *>(out) + (size_t)2 * FV * 16 + (size_t)2 * FL * 8);
    for (int mt = 0; mt < MTD; ++mt)
        for (int kt = 0; kt < KT; ++kt)
            for (int l = 0; l < 64; ++l) {
                const OutSlot o = out_slot(mt, l % 16);
                t32[(mt * KT + kt) * 64 + l] = (float)deriv_entry(N, D, o.g, o.s, 32 * KVS + 4 * kt + l / 16);
            }
    return (int)total;
}

}  // namespace dgw
