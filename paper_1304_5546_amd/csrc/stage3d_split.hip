// Fused LSRK stage for 3D Maxwell on tetrahedra with split-precision
// contractions: every operator product Op * b is evaluated as
//   Op_hi b_hi + Op_hi b_lo + Op_lo b_hi,   x_hi = bf16(x), x_lo = bf16(x - x_hi),
// on v_mfma_f32_16x16x32_bf16 with FP32 accumulation.  The right-hand side is
// the one of the FP32 3D kernel (3D analogue of eq. dg-strong-explicit):
//   1. D_p u for p = r, s, t and each of the six fields u (split MFMA; D_p
//      annihilates constants, so the operand is u - u(c) with c a node of the
//      element: the split then carries the variation across the element);
//   2. chain rule and curl in FP64 with the FP64 geometric factors
//      (eq. dg-diff-local-to-global);
//   3. upwind flux per face node in FP64 with the FP64 normals and surface
//      Jacobians (3D form of eq. max2d-numflux, factor 1/2), rounded to FP32;
//   4. LIFT of the flux (split MFMA) on top of the volume part, then the RK
//      update res <- a res + dt rhs, q_out <- q_in + b res (FP32 fields).
//
// Work unit = one wave and 16 elements as in the FP32 kernel; K walked in
// steps of 32 (lane group g holds rows 32 ks + 8 g + q, q = 0..7).  The
// hi/lo operator fragments sit in LDS.
#include <hip/hip_runtime.h>

#include "device.hpp"

namespace dgw {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

namespace {

template <int N>
struct TetS {
    static constexpr int Np = (N + 1) * (N + 2) * (N + 3) / 6;
    static constexpr int Nfp = (N + 1) * (N + 2) / 2;
    static constexpr int Nafp = 4 * Nfp;
    static constexpr int MT = (Np + 15) / 16;
    static constexpr int KV = (Np + 31) / 32;    // K-steps of a derivative
    static constexpr int KL = (Nafp + 31) / 32;  // K-steps of LIFT
    static constexpr int FV = 3 * MT * KV * 64;  // derivative fragments (uint4 per lane)
    static constexpr int FL = MT * KL * 64;      // LIFT fragments
    static constexpr int NT = Nafp + 4 * 6 * Nfp;
    static constexpr int CN = 0;  // the node whose value is taken out of the volume operand
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

}  // namespace

template <int N>
__global__ void __launch_bounds__(256, 2) stage3d_split_kernel(StageArgs A) {
    using T = TetS<N>;
    constexpr int Np = T::Np, Nfp = T::Nfp, Nafp = T::Nafp, MT = T::MT, KV = T::KV, KL = T::KL;
    constexpr int FV = T::FV, FL = T::FL, NT = T::NT;
    __shared__ uint4 sA[2 * (FV + FL)];  // hi fragments, then lo fragments
    __shared__ int stab[NT];
    // per wave: the face records and FP64 face data (n, Fscale) of its 16
    // elements, read per face node from LDS instead of memory
    __shared__ double sfd[4][4][4][16];
    __shared__ int srec[4][4][16];

    {
        const uint4 *src = reinterpret_cast<const uint4 *>(A.opsfrag);
        for (int i = threadIdx.x; i < 2 * (FV + FL); i += 256) sA[i] = src[i];
        for (int i = threadIdx.x; i < NT; i += 256) stab[i] = A.itab[i];
    }
    __syncthreads();

    const int lane0 = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int nu = 4 * A.ntiles;
    const int x = blockIdx.x & 7, bi = blockIdx.x >> 3, GB = gridDim.x >> 3;
    const int q8 = nu >> 3, r8 = nu & 7;
    const int xbase = x * q8 + (x < r8 ? x : r8), xcount = q8 + (x < r8 ? 1 : 0);
    const double halpha = 0.5 * (double)A.alpha;

    for (int ul = 4 * bi + w; ul < xcount; ul += 4 * GB) {
        const int u = xbase + ul;
        const int tile = u >> 2;
        int lane = lane0;
        asm volatile("" : "+v"(lane));
        const int g = lane >> 4, c = lane & 15;
        const int col = 16 * (u & 3) + c;
        constexpr unsigned TB = 6 * Np * 64 * 4;
        const __amdgpu_buffer_rsrc_t rq = rsrc(A.qin + (size_t)tile * (6 * Np * 64), TB);
        const unsigned vcol = (unsigned)col * 4;
        const unsigned vrow8 = (unsigned)(8 * g * 64 + col) * 4;  // row 32 ks + 8 g (+ q) of a K-step

        double G[9];
        {
            const double *gt = A.geo64 + (size_t)tile * (9 * 64);
#pragma unroll
            for (int q = 0; q < 9; ++q) G[q] = gt[(unsigned)(q * 64 + col)];
        }

        float cv[6][MT][4];
#pragma unroll
        for (int f = 0; f < 6; ++f)
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                for (int jj = 0; jj < 4; ++jj) cv[f][mt][jj] = 0.f;

        // ---- volume.  The next field's operand rows are in flight while the
        // current field is contracted; rows past Np meet zero operator
        // columns (values past the tile read as 0)
        float vn[KV][8], qcn = bload(rq, vcol, (0 * Np + T::CN) * 256);
#pragma unroll
        for (int ks = 0; ks < KV; ++ks)
#pragma unroll
            for (int q = 0; q < 8; ++q) vn[ks][q] = bload(rq, vrow8, (0 * Np + 32 * ks + q) * 256);
#pragma unroll
        for (int f = 0; f < 6; ++f) {
            float vc[KV][8];
            const float qc = qcn;
#pragma unroll
            for (int ks = 0; ks < KV; ++ks)
#pragma unroll
                for (int q = 0; q < 8; ++q) vc[ks][q] = vn[ks][q];
            if (f + 1 < 6) {
                qcn = bload(rq, vcol, ((f + 1) * Np + T::CN) * 256);
#pragma unroll
                for (int ks = 0; ks < KV; ++ks)
#pragma unroll
                    for (int q = 0; q < 8; ++q) vn[ks][q] = bload(rq, vrow8, ((f + 1) * Np + 32 * ks + q) * 256);
            }
            floatx4 d[3][MT];
#pragma unroll
            for (int p = 0; p < 3; ++p)
#pragma unroll
                for (int mt = 0; mt < MT; ++mt) d[p][mt] = floatx4{0.f, 0.f, 0.f, 0.f};
            int la = lane;
            asm volatile("" : "+v"(la));
#pragma unroll
            for (int ks = 0; ks < KV; ++ks) {
                bf16x8 bh, bl;
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    const float v = vc[ks][q] - qc;
                    const __bf16 h = (__bf16)v;
                    bh[q] = h;
                    bl[q] = (__bf16)(v - (float)h);
                }
#pragma unroll
                for (int p = 0; p < 3; ++p)
#pragma unroll
                    for (int mt = 0; mt < MT; ++mt) {
                        const int fi = ((p * MT + mt) * KV + ks) * 64 + la;
                        d[p][mt] = mfma3(as_bf16x8(sA[fi]), as_bf16x8(sA[FV + FL + fi]), bh, bl, d[p][mt]);
                    }
            }
            // chain rule and curl in FP64
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                for (int jj = 0; jj < 4; ++jj) {
                    const double dr = d[0][mt][jj], ds = d[1][mt][jj], dtt = d[2][mt][jj];
                    const double gx = G[0] * dr + G[3] * ds + G[6] * dtt;
                    const double gy = G[1] * dr + G[4] * ds + G[7] * dtt;
                    const double gz = G[2] * dr + G[5] * ds + G[8] * dtt;
                    if (f == 0) { cv[4][mt][jj] += (float)gz; cv[5][mt][jj] -= (float)gy; }
                    if (f == 1) { cv[3][mt][jj] -= (float)gz; cv[5][mt][jj] += (float)gx; }
                    if (f == 2) { cv[3][mt][jj] += (float)gy; cv[4][mt][jj] -= (float)gx; }
                    if (f == 3) { cv[1][mt][jj] -= (float)gz; cv[2][mt][jj] += (float)gy; }
                    if (f == 4) { cv[0][mt][jj] += (float)gz; cv[2][mt][jj] -= (float)gx; }
                    if (f == 5) { cv[0][mt][jj] -= (float)gy; cv[1][mt][jj] += (float)gx; }
                }
#pragma unroll
            for (int o = 0; o < 6; ++o)
#pragma unroll
                for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                    for (int jj = 0; jj < 4; ++jj) asm volatile("" : "+v"(cv[o][mt][jj]));
            __builtin_amdgcn_sched_barrier(0);
        }

        // ---- surface
        const __amdgpu_buffer_rsrc_t rn = rsrc(A.nbr + (size_t)tile * (4 * 64), 4 * 64 * 4);
        const __amdgpu_buffer_rsrc_t rall = rsrc(A.qin, (unsigned)A.ntiles * TB);
        {
            // lane group g fetches face g of its column
            const double *ft = A.fgeo64 + (size_t)tile * (16 * 64);
#pragma unroll
            for (int q = 0; q < 4; ++q) sfd[w][g][q][c] = ft[(unsigned)((4 * g + q) * 64 + col)];
            srec[w][g][c] = __builtin_bit_cast(int, bload(rn, vcol, g * 256));
        }
        floatx4 acc[6][MT];
#pragma unroll
        for (int f = 0; f < 6; ++f)
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
                acc[f][mt] = floatx4{cv[f][mt][0], cv[f][mt][1], cv[f][mt][2], cv[f][mt][3]};
        // own and partner traces of face-node slot t = 8 ks + q (node
        // j = 32 ks + 8 g + q), gathered RING - 1 slots ahead of their use.
        // RING = 1 (no slot ahead) keeps the kernel within its 256
        // registers; with a slot ahead registers spill and the order-4 stage
        // runs 1.4 % slower
        auto gather = [&](int t, float (&m)[6], float (&pv)[6], int &wall) {
            const int j = 32 * (t >> 3) + 8 * g + (t & 7);
            const int jc = j < Nafp ? j : Nafp - 1;
            const int face = jc / Nfp, i = jc - face * Nfp;
            const int own = stab[jc];
            const int rc = srec[w][face][c];
            wall = rc < 0;
            const int e2 = wall ? tile * 64 + col : (rc >> 5);
            const int pn = wall ? own : stab[Nafp + (((rc >> 3) & 3) * 6 + (rc & 7)) * Nfp + i];
            const unsigned vp = (((unsigned)(e2 >> 6) * (6 * Np) + pn) * 64 + (e2 & 63)) * 4;
            const unsigned vo = (unsigned)(own * 64 + col) * 4;
#pragma unroll
            for (int f = 0; f < 6; ++f) {
                m[f] = bload(rq, vo, f * Np * 256);
                pv[f] = bload(rall, vp, f * Np * 256);
            }
        };
        constexpr int NS = 8 * KL, RING = 1;
        float rm[RING][6], rp[RING][6];
        int rw[RING];
#pragma unroll
        for (int t = 0; t < RING - 1; ++t)
            if (t < NS) gather(t, rm[t], rp[t], rw[t]);
#pragma unroll
        for (int ks = 0; ks < KL; ++ks) {
            bf16x8 bh[6], bl[6];
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const int t = 8 * ks + q;
                if (t + RING - 1 < NS) gather(t + RING - 1, rm[(t + RING - 1) % RING], rp[(t + RING - 1) % RING],
                                              rw[(t + RING - 1) % RING]);
                const int j = 32 * ks + 8 * g + q;
                const int jc = j < Nafp ? j : Nafp - 1;
                const int face = jc / Nfp;
                const bool wall = rw[t % RING] != 0;
                double dq[6];
#pragma unroll
                for (int f = 0; f < 6; ++f) {
                    const double m = rm[t % RING][f], pv = rp[t % RING][f];
                    dq[f] = m - ((wall && f >= 3) ? -pv : pv);
                }
                const double nx = sfd[w][face][0][c], ny = sfd[w][face][1][c];
                const double nz = sfd[w][face][2][c], fs = sfd[w][face][3][c];
                const double dHx = dq[0], dHy = dq[1], dHz = dq[2], dEx = dq[3], dEy = dq[4], dEz = dq[5];
                const double ndH = nx * dHx + ny * dHy + nz * dHz;
                const double ndE = nx * dEx + ny * dEy + nz * dEz;
                const double h = j < Nafp ? 0.5 * fs : 0.0, ah = j < Nafp ? halpha * fs : 0.0;
                const double cEx = ny * dEz - nz * dEy, cEy = nz * dEx - nx * dEz, cEz = nx * dEy - ny * dEx;
                const double cHx = ny * dHz - nz * dHy, cHy = nz * dHx - nx * dHz, cHz = nx * dHy - ny * dHx;
                float fl[6];
                fl[0] = (float)(h * cEx + ah * (nx * ndH - dHx));
                fl[1] = (float)(h * cEy + ah * (ny * ndH - dHy));
                fl[2] = (float)(h * cEz + ah * (nz * ndH - dHz));
                fl[3] = (float)(-h * cHx + ah * (nx * ndE - dEx));
                fl[4] = (float)(-h * cHy + ah * (ny * ndE - dEy));
                fl[5] = (float)(-h * cHz + ah * (nz * ndE - dEz));
#pragma unroll
                for (int f = 0; f < 6; ++f) {
                    const __bf16 hh = (__bf16)fl[f];
                    bh[f][q] = hh;
                    bl[f][q] = (__bf16)(fl[f] - (float)hh);
                }
            }
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) {
                const int fi = FV + (mt * KL + ks) * 64 + lane;
                const bf16x8 ah = as_bf16x8(sA[fi]), al = as_bf16x8(sA[FV + FL + fi]);
#pragma unroll
                for (int f = 0; f < 6; ++f) acc[f][mt] = mfma3(ah, al, bh[f], bl[f], acc[f][mt]);
            }
            __builtin_amdgcn_sched_barrier(0);
        }

        // ---- fused low-storage RK update
        const __amdgpu_buffer_rsrc_t rr = rsrc(A.res + (size_t)tile * (6 * Np * 64), TB);
        const __amdgpu_buffer_rsrc_t ro = rsrc(A.qout + (size_t)tile * (6 * Np * 64), TB);
        const unsigned vout = (unsigned)(4 * g * 64 + col) * 4;
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
                    qv[mt][jj] = bload(rq, vout, so);
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
    }
}

template <int N>
static hipError_t launch3d_split(const StageArgs &a, hipStream_t s) {
    if (!a.opsfrag || !a.itab || !a.qin || !a.qout || !a.res || !a.geo64 || !a.fgeo64 || !a.nbr || a.ntiles <= 0 ||
        a.ngroups < 8 || (a.ngroups & 7))
        return hipErrorInvalidValue;
    hipLaunchKernelGGL((stage3d_split_kernel<N>), dim3(a.ngroups), dim3(256), 0, s, a);
    return hipGetLastError();
}

template <int N>
static int occupancy3d_split() {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, stage3d_split_kernel<N>, 256, 0) != hipSuccess) return 1;
    return nb > 0 ? nb : 1;
}

hipError_t launch_stage3d_split(int N, const StageArgs &a, hipStream_t s) {
    switch (N) {
        case 1: return launch3d_split<1>(a, s);
        case 2: return launch3d_split<2>(a, s);
        case 3: return launch3d_split<3>(a, s);
        case 4: return launch3d_split<4>(a, s);
        default: return hipErrorInvalidValue;
    }
}

int blocks_per_cu_3d_split(int N) {
    switch (N) {
        case 1: return occupancy3d_split<1>();
        case 2: return occupancy3d_split<2>();
        case 3: return occupancy3d_split<3>();
        case 4: return occupancy3d_split<4>();
        default: return 1;
    }
}

// Split operator fragments of the 3D split kernel, hi part then lo part,
// each [Dr, Ds, Dt blocks: (p, mt, ks)][LIFT: (mt, ks)] x 64 lanes x 8 BF16:
// lane l of block (mt, ks) holds M[16 mt + l%16][32 ks + 8 (l/16) + q].
// Returns the size in bytes (out == nullptr: size only).
static uint16_t bf16_bits(float f) {
    uint32_t u;
    __builtin_memcpy(&u, &f, 4);
    return (uint16_t)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);  // nearest even (finite inputs)
}
static float bf16_value(uint16_t h) {
    const uint32_t u = (uint32_t)h << 16;
    float f;
    __builtin_memcpy(&f, &u, 4);
    return f;
}

int opsfrag3d_split(int N, const double *Dr, const double *Ds, const double *Dt, const double *LIFT, void *out) {
    const int Np = (N + 1) * (N + 2) * (N + 3) / 6, Nafp = 4 * ((N + 1) * (N + 2) / 2);
    const int MT = (Np + 15) / 16, KV = (Np + 31) / 32, KL = (Nafp + 31) / 32;
    const int FV = 3 * MT * KV * 64, FL = MT * KL * 64;
    const size_t total = (size_t)2 * (FV + FL) * 16;
    if (!out) return (int)total;
    uint16_t *o = static_cast<uint16_t *>(out);
    const size_t lo_off = (size_t)(FV + FL) * 8;
    auto put = [&](size_t frag, const double *M, int cols, int mt, int ks, int l) {
        for (int q = 0; q < 8; ++q) {
            const int row = 16 * mt + (l % 16), k = 32 * ks + 8 * (l / 16) + q;
            const double v = (row < Np && k < cols) ? M[(size_t)row * cols + k] : 0.0;
            const uint16_t hi = bf16_bits((float)v);
            const uint16_t lo = bf16_bits((float)(v - (double)bf16_value(hi)));
            o[frag * 8 + q] = hi;
            o[lo_off + frag * 8 + q] = lo;
        }
    };
    const double *D[3] = {Dr, Ds, Dt};
    for (int p = 0; p < 3; ++p)
        for (int mt = 0; mt < MT; ++mt)
            for (int ks = 0; ks < KV; ++ks)
                for (int l = 0; l < 64; ++l) put((size_t)((p * MT + mt) * KV + ks) * 64 + l, D[p], Np, mt, ks, l);
    for (int mt = 0; mt < MT; ++mt)
        for (int ks = 0; ks < KL; ++ks)
            for (int l = 0; l < 64; ++l) put((size_t)FV + (mt * KL + ks) * 64 + l, LIFT, Nafp, mt, ks, l);
    return (int)total;
}

}  // namespace dgw
