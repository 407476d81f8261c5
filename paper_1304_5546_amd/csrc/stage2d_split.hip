// Fused LSRK stage for 2D TM Maxwell with split-precision contractions on the
// matrix cores of gfx950 (v_mfma_f32_16x16x32_{bf16,f16}).
//
// Same right-hand side and fused operator as the FP32 MFMA kernel
// (Op = [Dr | Ds | LIFT], one contraction per output field, eq.
// dg-strong-explicit), but every product Op * B is evaluated as
//   A_hi B_hi + A_hi B_lo + A_lo B_hi,    X_hi = round16(X), X_lo = round16(X - X_hi),
// with 16-bit BF16 (8-bit significand) or FP16 (11-bit) parts and FP32
// accumulation.  A_hi/A_lo are split once on the host from the FP64 operator;
// B_hi/B_lo are split per K-step from the FP32 operand.  The geometric
// factors (r_x, r_y, s_x, s_y), normals and surface Jacobians stay FP64 on
// the GPU: the volume operand g*(q - q_c) (q_c a per-element constant, see
// below) and the flux are formed in FP64 and rounded once to FP32 before the
// split.
//
// Structure as the FP32 kernel: persistent, warp-specialised (4 producer
// waves stream the next 64-element tile's fields and partner traces into a
// double-buffered LDS tile; 4 consumer waves each own a 16-element MFMA
// N-tile), K walked in steps of 32 (lane group g holds 8 consecutive K rows).
#include <hip/hip_runtime.h>

#include <cstdint>

#include "device.hpp"

namespace dgw {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 halfx8 __attribute__((ext_vector_type(8)));

namespace {

template <int PREC>
struct P16;
template <>
struct P16<1> {  // BF16
    typedef __bf16 T;
    typedef bf16x8 V;
    __device__ static floatx4 mfma(V a, V b, floatx4 c) { return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0); }
};
template <>
struct P16<2> {  // FP16
    typedef _Float16 T;
    typedef halfx8 V;
    __device__ static floatx4 mfma(V a, V b, floatx4 c) { return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0); }
};

template <int N, bool MAT>
struct TriS {
    static constexpr int Np = (N + 1) * (N + 2) / 2;
    static constexpr int Nfp = N + 1;
    static constexpr int Nafp = 3 * Nfp;
    static constexpr int KV = (Np + 31) / 32;    // K-steps of 32 of a derivative
    static constexpr int KF = (Nafp + 31) / 32;  // K-steps of 32 of LIFT
    static constexpr int MT = (Np + 15) / 16;
    static constexpr int FV = 2 * MT * KV * 64;  // Dr, Ds fragments (uint4 = 8 x 16 bit per lane)
    static constexpr int FA = FV + MT * KF * 64; // + LIFT fragments: offset of the lo parts
    static constexpr int G = MAT ? 6 : 4;
    static constexpr int FG = MAT ? 6 : 3;
    static constexpr int RP = 3 * Np;          // partner traces / flux rows
    static constexpr int R = RP + 3 * Nafp;
    static constexpr int SUB = R * 16 + ((R & 1) ? 0 : 16);
    static constexpr int BUF = 4 * SUB;
    static constexpr int JW = (Nafp + 3) / 4;
    __host__ __device__ static constexpr int lat(int i, int j) { return j * (N + 1) - j * (j - 1) / 2 + i; }
    __host__ __device__ static constexpr int face_node(int f, int t) {
        return f == 0 ? t : (f == 1 ? lat(N - t, t) : lat(0, N - t));
    }
};

// Op_hi b_hi + Op_hi b_lo + Op_lo b_hi accumulated on c.
template <int PREC>
__device__ __forceinline__ floatx4 mfma3(uint4 ahu, uint4 alu, typename P16<PREC>::V bh, typename P16<PREC>::V bl,
                                         floatx4 c) {
    typename P16<PREC>::V ah, al;
    __builtin_memcpy(&ah, &ahu, 16);
    __builtin_memcpy(&al, &alu, 16);
    c = P16<PREC>::mfma(ah, bh, c);
    c = P16<PREC>::mfma(ah, bl, c);
    return P16<PREC>::mfma(al, bh, c);
}

// Maximum of x over the four lanes l, l ^ 16, l ^ 32, l ^ 48 (the four lane
// groups of a column).  A row swap of x with itself hands each row of 16
// lanes its partner row's values (16-lane rows paired within each half,
// then the two halves), on the VALU rather than through the LDS crossbar.
__device__ __forceinline__ float col_max(float x) {
    const unsigned u = __float_as_uint(x);
    const auto r16 = __builtin_amdgcn_permlane16_swap(u, u, false, false);
    x = fmaxf(__uint_as_float(r16[0]), __uint_as_float(r16[1]));
    const unsigned v = __float_as_uint(x);
    const auto r32 = __builtin_amdgcn_permlane32_swap(v, v, false, false);
    return fmaxf(__uint_as_float(r32[0]), __uint_as_float(r32[1]));
}

// Power-of-two scale taking a column maximum mx (per lane group) below 2^14,
// reduced over the four lane groups of the column.
__device__ __forceinline__ void pow2_scale(float mx, float &scale, float &unscale) {
    mx = col_max(mx);
    scale = unscale = 1.f;
    if (mx > 0.f && mx < 3.0e38f) {
        int ex;
        frexpf(mx, &ex);  // mx < 2^ex
        scale = ldexpf(1.f, 14 - ex);
        unscale = ldexpf(1.f, ex - 14);
    }
}

}  // namespace

// Producer pause (units of 64 cycles) at the top of each tile, so that the
// consumers' loads are issued ahead of the producers' stream.
#ifndef DGW_SP_PSLEEP
#define DGW_SP_PSLEEP 0
#endif
// Consumers load their FP64 factors and face data one tile ahead (1), and
// their residual rows at tile start instead of one tile ahead (1).
#ifndef DGW_SP_GPF
#define DGW_SP_GPF 1
#endif
#ifndef DGW_SP_RSTART
#define DGW_SP_RSTART 0
#endif
// Where in the tile the next tile's prefetches are issued: 0 after the
// update, 1 before it, 2 at tile start.
#ifndef DGW_SP_PFAT
#define DGW_SP_PFAT 1
#endif

template <int N, bool MAT, int PREC>
__global__ void __launch_bounds__(512) stage2d_split_kernel(StageArgs A) {
    using T = TriS<N, MAT>;
    using H = P16<PREC>;
    typedef typename H::T h16;
    typedef typename H::V hv;
    constexpr int Np = T::Np, Nfp = T::Nfp, Nafp = T::Nafp, KV = T::KV, KF = T::KF, MT = T::MT;
    constexpr int FV = T::FV, FA = T::FA;
    constexpr int G = T::G, FG = T::FG, RP = T::RP, SUB = T::SUB, BUF = T::BUF, JW = T::JW;
    __shared__ float sbuf[2 * BUF];
    __shared__ uint4 sa[2 * FA];  // operator fragments: hi parts, then lo parts

    const int lane0 = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const bool producer = wv >= 4;
    const int w = wv & 3;

    {
        const uint4 *src = reinterpret_cast<const uint4 *>(A.opsfrag);
        for (int i = threadIdx.x; i < 2 * FA; i += 512) sa[i] = src[i];
    }

    const int x = blockIdx.x & 7, bi = blockIdx.x >> 3, GB = gridDim.x >> 3;
    const int q8 = A.ntiles >> 3, r8 = A.ntiles & 7;
    const int xbase = x * q8 + (x < r8 ? x : r8), xcount = q8 + (x < r8 ? 1 : 0);
    if (bi >= xcount) return;

    const int prow = (lane0 >> 4) * SUB + (lane0 & 15);
    int rec_next[3] = {-1, -1, -1};
    auto load_recs = [&](int tile) {
        const int *nt = A.nbr + (size_t)tile * (3 * 64);
        int ln = lane0;
        asm volatile("" : "+v"(ln));
#pragma unroll
        for (int f = 0; f < 3; ++f) rec_next[f] = nt[(unsigned)(f * 64 + ln)];
    };
    auto produce = [&](int tile, int b) {
        const float *qt = A.qin + (size_t)tile * (3 * Np * 64);
        int rec[3] = {rec_next[0], rec_next[1], rec_next[2]};
        int ln = lane0;
        asm volatile("" : "+v"(ln));
        // field rows in quads of 4 rows x 64 elements, one 16-byte access per
        // lane: lane l takes row 4 quad + l/16, elements 4 (l%16) .. + 3;
        // producer w takes quads w, w + 4, ...
        constexpr int PV = ((RP + 3) / 4 + 3) / 4;
        floatx4 pv[PV];
        const int lr = ln >> 4, le = 4 * (ln & 15);
#pragma unroll
        for (int i = 0; i < PV; ++i) {
            const int r = 4 * (w + 4 * i) + lr;
            pv[i] = r < RP ? *reinterpret_cast<const floatx4 *>(qt + (unsigned)(r * 64 + le)) : floatx4{0.f, 0.f, 0.f, 0.f};
        }
        float pt[JW][3];
#pragma unroll
        for (int i = 0; i < JW; ++i) {
            const int j = w + 4 * i;
            pt[i][0] = pt[i][1] = pt[i][2] = 0.f;
            if (j < Nafp) {
                const int face = j / Nfp, t = j - face * Nfp;
                const int rc = rec[face];
                const bool wall = rc < 0;
                const int e2 = wall ? tile * 64 + ln : (rc >> 5);
                const int pn = wall ? T::face_node(face, t) : T::face_node((rc >> 3) & 3, (rc & 7) ? N - t : t);
                const unsigned i0 = ((unsigned)(e2 >> 6) * (3 * Np) + pn) * 64 + (e2 & 63);
#pragma unroll
                for (int f = 0; f < 3; ++f) pt[i][f] = A.qin[i0 + f * Np * 64];
                if (wall) pt[i][2] = -pt[i][2];  // PEC mirror: Ez+ = -Ez-, H+ = H-
            }
        }
        float *Bp = sbuf + b * BUF + prow;
        // element 4 (l%16) + q of a quad row lies in sub-tile (l%16)/4, column 4 (l%4) + q
        float *Bv = sbuf + b * BUF + ((ln & 15) >> 2) * SUB + 4 * (ln & 3);
#pragma unroll
        for (int i = 0; i < PV; ++i) {
            const int r = 4 * (w + 4 * i) + lr;
            if (r < RP) *reinterpret_cast<floatx4 *>(Bv + r * 16) = pv[i];
        }
#pragma unroll
        for (int i = 0; i < JW; ++i) {
            const int j = w + 4 * i;
            if (j < Nafp) {
#pragma unroll
                for (int f = 0; f < 3; ++f) Bp[(RP + f * Nafp + j) * 16] = pt[i][f];
            }
        }
    };

    if (producer) {
        load_recs(xbase + bi);
        produce(xbase + bi, 0);
        if (bi + GB < xcount) load_recs(xbase + bi + GB);
    }
    __syncthreads();

    // consumers: the residual rows of their next tile are loaded at the end of
    // the current one, so the update never waits on memory.  Consumer memory
    // traffic is row-major and 16 bytes wide: lane l covers field rows
    // 16 rg + l/4 and, of the wave's 16 elements, the columns 4 (l%4) .. + 3;
    // the right-hand side is transposed to that order through the wave's own
    // LDS sub-tile at the update (3 RGN vector-memory instructions per tile)
    constexpr int RGN = (3 * Np + 15) / 16;
    floatx4 rrn[RGN];
    auto load_res = [&](int tile) {
        int ln = lane0;
        asm volatile("" : "+v"(ln));
        const float *rt = A.res + (size_t)tile * (3 * Np * 64) + 16 * w + 4 * (ln & 3);
#pragma unroll
        for (int rg = 0; rg < RGN; ++rg) {
            const int row = 16 * rg + (ln >> 2);
            rrn[rg] = row < 3 * Np ? *reinterpret_cast<const floatx4 *>(rt + (unsigned)(row * 64))
                                   : floatx4{0.f, 0.f, 0.f, 0.f};
        }
    };
    // The factor prefetch and the early placement cost registers: below
    // order 6 (where two work-groups share a CU) both are off, and the
    // material forms and order 8 keep the prefetches at the end of the tile.
    constexpr bool GPF = DGW_SP_GPF && N >= 6;
    constexpr int PFAT = (MAT || N > 7 || N < 6) ? 0 : DGW_SP_PFAT;
    // FP64 geometric factors and face data of the lane's element (with
    // GPF loaded one tile ahead, at the end of the previous tile)
    double gdn[G], fdn[3][FG];
    auto load_geo = [&](int tile) {
        int ln = lane0;
        asm volatile("" : "+v"(ln));
        const int col = 16 * w + (ln & 15);
        const double *gt = A.geo64 + (size_t)tile * (G * 64);
#pragma unroll
        for (int q = 0; q < G; ++q) gdn[q] = gt[q * 64 + col];
        const double *ft = A.fgeo64 + (size_t)tile * (3 * FG * 64);
#pragma unroll
        for (int f = 0; f < 3; ++f)
#pragma unroll
            for (int q = 0; q < FG; ++q) fdn[f][q] = ft[(f * FG + q) * 64 + col];
    };
    if (!producer) {
        if (!DGW_SP_RSTART) load_res(xbase + bi);
        if (GPF) load_geo(xbase + bi);
    }

    // Producer and consumer waves run separate tile loops with the same
    // (wave-uniform) trip count and one barrier per tile each (the barrier
    // counts waves, not program locations): with one loop and a role branch
    // inside, the roles' register state would join at the barrier and the
    // compiler would copy the consumers' in-flight prefetch registers there,
    // waiting for the loads.
    if (producer) {
        int it = 0;
        for (int tl = bi; tl < xcount; tl += GB, ++it) {
            const int cur = it & 1;
            const int tn = tl + GB;
            if (DGW_SP_PSLEEP > 0) __builtin_amdgcn_s_sleep(DGW_SP_PSLEEP);
            if (tn < xcount) {
                produce(xbase + tn, cur ^ 1);
                if (tn + GB < xcount) load_recs(xbase + tn + GB);
            }
            __syncthreads();
        }
    } else {
        int it = 0;
        for (int tl = bi; tl < xcount; tl += GB, ++it) {
            const int cur = it & 1;
            const int tile = xbase + tl;
            int lane = lane0;
            asm volatile("" : "+v"(lane));
            const int g = lane >> 4, c = lane & 15;
            const int col = 16 * w + c;
            float *B = sbuf + cur * BUF + w * SUB + c;
            float *rt = A.res + (size_t)tile * (3 * Np * 64);
            float *ot = A.qout + (size_t)tile * (3 * Np * 64);

            if (DGW_SP_RSTART) load_res(tile);
            floatx4 rr[RGN];
#pragma unroll
            for (int rg = 0; rg < RGN; ++rg) rr[rg] = rrn[rg];
            // FP64 geometric factors and face data of column col
            if (!GPF) load_geo(tile);
            double gd[G], fd[3][FG];
#pragma unroll
            for (int q = 0; q < G; ++q) gd[q] = gdn[q];
#pragma unroll
            for (int f = 0; f < 3; ++f)
#pragma unroll
                for (int q = 0; q < FG; ++q) fd[f][q] = fdn[f][q];
            if (PFAT == 2) {
                // unconditional (the last tile re-reads its own data, unused):
                // a conditional prefetch makes the compiler copy the
                // loop-carried registers, waiting for the loads
                const int tp = xbase + (tl + GB < xcount ? tl + GB : tl);
                if (!DGW_SP_RSTART) load_res(tp);
                if (GPF) load_geo(tp);
            }
            const double rx = gd[0], ry = gd[1], sx = gd[2], sy = gd[3];
            double ieps = 1.0, imu = 1.0;
            if (MAT) {
                ieps = gd[4 % G];
                imu = gd[5 % G];
            }

            // upwind flux of this wave's 16 elements (FP64 coefficients), in place
#pragma unroll
            for (int jb = 0; jb < (Nafp + 3) / 4; ++jb) {
                const int j = 4 * jb + g;
                if (j < Nafp) {
                    const int face = j / Nfp, t = j - face * Nfp;
                    const int own = T::face_node(face, t);
                    const double dHx = (double)B[(0 * Np + own) * 16] - (double)B[(RP + 0 * Nafp + j) * 16];
                    const double dHy = (double)B[(1 * Np + own) * 16] - (double)B[(RP + 1 * Nafp + j) * 16];
                    const double dEz = (double)B[(2 * Np + own) * 16] - (double)B[(RP + 2 * Nafp + j) * 16];
                    double v[FG];
#pragma unroll
                    for (int q = 0; q < FG; ++q) v[q] = face == 0 ? fd[0][q] : face == 1 ? fd[1][q] : fd[2][q];
                    const double nx = v[0], ny = v[1];
                    const double dh = nx * dHy - ny * dHx;
                    double cEE, cEh, cHE, cHh;
                    if (MAT) {
                        cEE = v[2];
                        cEh = v[3 % FG];
                        cHE = v[4 % FG];
                        cHh = v[5 % FG];
                    } else {
                        const double hs = 0.5 * v[2];
                        cEE = (double)A.alpha * hs;
                        cEh = hs;
                        cHE = hs;
                        cHh = (double)A.alpha * hs;
                    }
                    const double fE = -(cEE * dEz + cEh * dh);
                    const double fH = cHE * dEz + cHh * dh;
                    B[(RP + 0 * Nafp + j) * 16] = (float)(ny * fH);
                    B[(RP + 1 * Nafp + j) * 16] = (float)(-nx * fH);
                    B[(RP + 2 * Nafp + j) * 16] = (float)fE;
                }
            }

            // ---- volume: D_r u and D_s u of each source field u by split
            // MFMA (K-steps of 32, lane group g holds rows 32 ks + 8 g + q),
            // then the chain rule and curl in FP64 on the results.  Dr and Ds
            // annihilate constants, so the operand is u - u(c), c a node near
            // the centroid: the split then carries the variation across the
            // element (small for resolved fields) rather than the field.
            constexpr int CN = T::lat(N / 3, N / 3);
            float cv[3][MT][4];
#pragma unroll
            for (int f = 0; f < 3; ++f)
#pragma unroll
                for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                    for (int jj = 0; jj < 4; ++jj) cv[f][mt][jj] = 0.f;
#pragma unroll
            for (int sf = 0; sf < 3; ++sf) {  // Hx, Hy, Ez
                const float uc = B[(sf * Np + CN) * 16];
                // FP16 (5-bit exponent): scale the operand column by a power of
                // two so that its largest entry is below 2^14, undo it exactly;
                // the column maximum is taken over the lane's own operand
                // entries (K row 32 ks + 8 g + q), read once for both uses
                float vr[KV][8];
                float scale = 1.f, unscale = 1.f;
                if constexpr (PREC == 2) {
#pragma unroll
                    for (int ks = 0; ks < KV; ++ks)
#pragma unroll
                        for (int q = 0; q < 8; ++q) {
                            const int k = 32 * ks + 8 * g + q;
                            vr[ks][q] = k < Np ? B[(sf * Np + k) * 16] - uc : 0.f;
                        }
                    float mx = 0.f;
#pragma unroll
                    for (int ks = 0; ks < KV; ++ks)
#pragma unroll
                        for (int q = 0; q < 8; ++q) mx = fmaxf(mx, fabsf(vr[ks][q]));
                    pow2_scale(mx, scale, unscale);
                }
                floatx4 d[2][MT];
#pragma unroll
                for (int p = 0; p < 2; ++p)
#pragma unroll
                    for (int mt = 0; mt < MT; ++mt) d[p][mt] = floatx4{0.f, 0.f, 0.f, 0.f};
                int la = lane;
                asm volatile("" : "+v"(la));
#pragma unroll
                for (int ks = 0; ks < KV; ++ks) {
                    hv bh, bl;
#pragma unroll
                    for (int q = 0; q < 8; ++q) {
                        float v;
                        if constexpr (PREC == 2) {
                            v = vr[ks][q] * scale;
                        } else {
                            const int k = 32 * ks + 8 * g + q;
                            v = k < Np ? B[(sf * Np + k) * 16] - uc : 0.f;
                        }
                        const h16 hi = (h16)v;
                        bh[q] = hi;
                        bl[q] = (h16)(v - (float)hi);
                    }
#pragma unroll
                    for (int p = 0; p < 2; ++p)
#pragma unroll
                        for (int mt = 0; mt < MT; ++mt) {
                            const int fi = ((p * MT + mt) * KV + ks) * 64 + la;
                            d[p][mt] = mfma3<PREC>(sa[fi], sa[FA + fi], bh, bl, d[p][mt]);
                        }
                }
#pragma unroll
                for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                    for (int jj = 0; jj < 4; ++jj) {
                        const double dr = (double)(d[0][mt][jj] * unscale), ds = (double)(d[1][mt][jj] * unscale);
                        const double dx = rx * dr + sx * ds, dy = ry * dr + sy * ds;
                        if (sf == 0) cv[2][mt][jj] -= (float)(ieps * dy);  // Ez -= dy Hx / eps
                        if (sf == 1) cv[2][mt][jj] += (float)(ieps * dx);  // Ez += dx Hy / eps
                        if (sf == 2) {
                            cv[0][mt][jj] -= (float)(imu * dy);  // Hx -= dy Ez / mu
                            cv[1][mt][jj] += (float)(imu * dx);  // Hy += dx Ez / mu
                        }
                    }
                // materialise the sums here (not sunk to the update)
#pragma unroll
                for (int o = 0; o < 3; ++o)
#pragma unroll
                    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                        for (int jj = 0; jj < 4; ++jj) asm volatile("" : "+v"(cv[o][mt][jj]));
                __builtin_amdgcn_sched_barrier(0);
            }

            // ---- LIFT of the flux rows (split MFMA), on top of the volume part
            floatx4 acc[3][MT];
#pragma unroll
            for (int f = 0; f < 3; ++f) {
                float vr[KF][8];
                float scale = 1.f, unscale = 1.f;
                if constexpr (PREC == 2) {
#pragma unroll
                    for (int ks = 0; ks < KF; ++ks)
#pragma unroll
                        for (int q = 0; q < 8; ++q) {
                            const int k = 32 * ks + 8 * g + q;
                            vr[ks][q] = k < Nafp ? B[(RP + f * Nafp + k) * 16] : 0.f;
                        }
                    float mx = 0.f;
#pragma unroll
                    for (int ks = 0; ks < KF; ++ks)
#pragma unroll
                        for (int q = 0; q < 8; ++q) mx = fmaxf(mx, fabsf(vr[ks][q]));
                    pow2_scale(mx, scale, unscale);
                }
                floatx4 t[MT];
#pragma unroll
                for (int mt = 0; mt < MT; ++mt) t[mt] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int ks = 0; ks < KF; ++ks) {
                    hv bh, bl;
#pragma unroll
                    for (int q = 0; q < 8; ++q) {
                        float v;
                        if constexpr (PREC == 2) {
                            v = vr[ks][q] * scale;
                        } else {
                            const int k = 32 * ks + 8 * g + q;
                            v = k < Nafp ? B[(RP + f * Nafp + k) * 16] : 0.f;
                        }
                        const h16 hi = (h16)v;
                        bh[q] = hi;
                        bl[q] = (h16)(v - (float)hi);
                    }
#pragma unroll
                    for (int mt = 0; mt < MT; ++mt) {
                        const int fi = FV + (mt * KF + ks) * 64 + lane;
                        t[mt] = mfma3<PREC>(sa[fi], sa[FA + fi], bh, bl, t[mt]);
                    }
                }
#pragma unroll
                for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                    for (int jj = 0; jj < 4; ++jj) acc[f][mt][jj] = cv[f][mt][jj] + t[mt][jj] * unscale;
            }

            if (PFAT == 1) {
                // unconditional (the last tile re-reads its own data, unused):
                // a conditional prefetch makes the compiler copy the
                // loop-carried registers, waiting for the loads
                const int tp = xbase + (tl + GB < xcount ? tl + GB : tl);
                if (!DGW_SP_RSTART) load_res(tp);
                if (GPF) load_geo(tp);
            }
            // fused low-storage RK update, row-major: the lane's q_in rows are
            // read first, the right-hand side (rows 16mt+4g+jj of column c) is
            // written over the sub-tile's field rows and read back row-major
            // (LDS operations of one wave complete in order)
            float *Bs = B - c;
            const int lr = lane >> 2, lc = 4 * (lane & 3);
            floatx4 qv[RGN];
#pragma unroll
            for (int rg = 0; rg < RGN; ++rg) {
                const int row = 16 * rg + lr;
                qv[rg] = row < 3 * Np ? *reinterpret_cast<const floatx4 *>(Bs + row * 16 + lc) : floatx4{0.f, 0.f, 0.f, 0.f};
            }
#pragma unroll
            for (int f = 0; f < 3; ++f)
#pragma unroll
                for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                    for (int jj = 0; jj < 4; ++jj) {
                        const int n = 16 * mt + 4 * g + jj;
                        if (n < Np) B[(f * Np + n) * 16] = acc[f][mt][jj];
                    }
            float *rtl = rt + 16 * w + lc, *otl = ot + 16 * w + lc;
#pragma unroll
            for (int rg = 0; rg < RGN; ++rg) {
                const int row = 16 * rg + lr;
                if (row < 3 * Np) {
                    const floatx4 rh = *reinterpret_cast<const floatx4 *>(Bs + row * 16 + lc);
                    floatx4 r, qo;
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        r[q] = A.a * rr[rg][q] + A.dt * rh[q];
                        qo[q] = qv[rg][q] + A.b * r[q];
                    }
                    *reinterpret_cast<floatx4 *>(rtl + (unsigned)(row * 64)) = r;
                    *reinterpret_cast<floatx4 *>(otl + (unsigned)(row * 64)) = qo;
                }
            }
            if (PFAT == 0) {
                // unconditional (the last tile re-reads its own data, unused):
                // a conditional prefetch makes the compiler copy the
                // loop-carried registers, waiting for the loads
                const int tp = xbase + (tl + GB < xcount ? tl + GB : tl);
                if (!DGW_SP_RSTART) load_res(tp);
                if (GPF) load_geo(tp);
            }
            __syncthreads();
        }
    }
}

template <int N, bool MAT, int PREC>
static hipError_t launch2d_split_t(const StageArgs &a, hipStream_t s) {
    // every pointer the kernel dereferences must be set
    if (!a.opsfrag || !a.geo64 || !a.fgeo64 || !a.qin || !a.qout || !a.res || !a.nbr || a.ntiles <= 0 ||
        a.ngroups < 8 || (a.ngroups & 7))
        return hipErrorInvalidValue;
    hipLaunchKernelGGL((stage2d_split_kernel<N, MAT, PREC>), dim3(a.ngroups), dim3(512), 0, s, a);
    return hipGetLastError();
}

template <int N, bool MAT, int PREC>
static int occupancy2d_split_t() {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, stage2d_split_kernel<N, MAT, PREC>, 512, 0) != hipSuccess)
        return 1;
    return nb > 0 ? nb : 1;
}

#define DGW_SPLIT_SWITCH(FN, RET_DEFAULT)                                                             \
    switch (N * 4 + (material ? 2 : 0) + (prec == 2 ? 1 : 0)) {                                       \
        DGW_SPLIT_N(1) DGW_SPLIT_N(2) DGW_SPLIT_N(3) DGW_SPLIT_N(4) DGW_SPLIT_N(5) DGW_SPLIT_N(6)   \
        DGW_SPLIT_N(7) DGW_SPLIT_N(8) default : return RET_DEFAULT;                                  \
    }

hipError_t launch_stage2d_split(int N, bool material, int prec, const StageArgs &a, hipStream_t s) {
#define DGW_SPLIT_N(n)                                                  \
    case n * 4 + 0: return launch2d_split_t<n, false, 1>(a, s);         \
    case n * 4 + 1: return launch2d_split_t<n, false, 2>(a, s);         \
    case n * 4 + 2: return launch2d_split_t<n, true, 1>(a, s);          \
    case n * 4 + 3: return launch2d_split_t<n, true, 2>(a, s);
    DGW_SPLIT_SWITCH(launch, hipErrorInvalidValue)
#undef DGW_SPLIT_N
}

int blocks_per_cu_2d_split(int N, bool material, int prec) {
#define DGW_SPLIT_N(n)                                                  \
    case n * 4 + 0: return occupancy2d_split_t<n, false, 1>();          \
    case n * 4 + 1: return occupancy2d_split_t<n, false, 2>();          \
    case n * 4 + 2: return occupancy2d_split_t<n, true, 1>();           \
    case n * 4 + 3: return occupancy2d_split_t<n, true, 2>();
    DGW_SPLIT_SWITCH(occ, 1)
#undef DGW_SPLIT_N
}

// ---- host side: split the FP64 operator into 16-bit hi/lo A fragments

static uint16_t to_bf16_bits(float f) {
    uint32_t u;
    __builtin_memcpy(&u, &f, 4);
    if ((u & 0x7fffffffu) > 0x7f800000u) return 0x7fc0;  // NaN
    const uint32_t bias = 0x7fffu + ((u >> 16) & 1u);      // round to nearest even
    return (uint16_t)((u + bias) >> 16);
}
static float from_bf16_bits(uint16_t h) {
    const uint32_t u = (uint32_t)h << 16;
    float f;
    __builtin_memcpy(&f, &u, 4);
    return f;
}
static uint16_t to_f16_bits(float f) {
    _Float16 h = (_Float16)f;  // round to nearest even
    uint16_t b;
    __builtin_memcpy(&b, &h, 2);
    return b;
}
static float from_f16_bits(uint16_t b) {
    _Float16 h;
    __builtin_memcpy(&h, &b, 2);
    return (float)h;
}

// Operator fragments of the 2D split kernel, hi parts then lo parts, each
// [Dr blocks (mt, ks < KV)][Ds blocks][LIFT blocks (mt, ks < KF)] x 64 lanes
// x 8 values: lane l of block (mt, ks) holds M[16 mt + l%16][32 ks + 8 (l/16) + q]
// (zero outside M).  Returns the size in bytes (out == nullptr: size only).
int opsfrag2d_split(int N, int prec, const double *Dr, const double *Ds, const double *LIFT, void *out) {
    const int Np = (N + 1) * (N + 2) / 2, Nafp = 3 * (N + 1);
    const int MT = (Np + 15) / 16, KV = (Np + 31) / 32, KF = (Nafp + 31) / 32;
    const int FV = 2 * MT * KV * 64, FA = FV + MT * KF * 64;
    const size_t total = (size_t)2 * FA * 16;
    if (!out) return (int)total;
    uint16_t *o = static_cast<uint16_t *>(out);
    auto put = [&](size_t frag, const double *M, int cols, int mt, int ks, int l) {
        for (int q = 0; q < 8; ++q) {
            const int row = 16 * mt + (l % 16), k = 32 * ks + 8 * (l / 16) + q;
            const double v = (row < Np && k < cols) ? M[(size_t)row * cols + k] : 0.0;
            uint16_t hi, lo;
            if (prec == 1) {
                hi = to_bf16_bits((float)v);
                lo = to_bf16_bits((float)(v - (double)from_bf16_bits(hi)));
            } else {
                hi = to_f16_bits((float)v);
                lo = to_f16_bits((float)(v - (double)from_f16_bits(hi)));
            }
            o[frag * 8 + q] = hi;
            o[(size_t)FA * 8 + frag * 8 + q] = lo;
        }
    };
    const double *D[2] = {Dr, Ds};
    for (int p = 0; p < 2; ++p)
        for (int mt = 0; mt < MT; ++mt)
            for (int ks = 0; ks < KV; ++ks)
                for (int l = 0; l < 64; ++l) put((size_t)((p * MT + mt) * KV + ks) * 64 + l, D[p], Np, mt, ks, l);
    for (int mt = 0; mt < MT; ++mt)
        for (int ks = 0; ks < KF; ++ks)
            for (int l = 0; l < 64; ++l) put((size_t)FV + (mt * KF + ks) * 64 + l, LIFT, Nafp, mt, ks, l);
    return (int)total;
}

}  // namespace dgw
