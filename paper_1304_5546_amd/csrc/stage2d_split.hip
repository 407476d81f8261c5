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
    static constexpr int Kd = 2 * Np + Nafp;
    static constexpr int KS = (Kd + 31) / 32;  // K-steps of 32
    static constexpr int MT = (Np + 15) / 16;
    static constexpr int G = MAT ? 6 : 4;
    static constexpr int FG = MAT ? 6 : 3;
    static constexpr int RP = 3 * Np;          // partner traces / flux rows
    static constexpr int R = RP + 3 * Nafp;
    static constexpr int SUB = R * 16 + ((R & 1) ? 0 : 16);
    static constexpr int BUF = 4 * SUB;
    static constexpr int QW = (RP + 3) / 4;
    static constexpr int JW = (Nafp + 3) / 4;
    __host__ __device__ static constexpr int lat(int i, int j) { return j * (N + 1) - j * (j - 1) / 2 + i; }
    __host__ __device__ static constexpr int face_node(int f, int t) {
        return f == 0 ? t : (f == 1 ? lat(N - t, t) : lat(0, N - t));
    }
};

}  // namespace

template <int N, bool MAT, int PREC>
__global__ void __launch_bounds__(512) stage2d_split_kernel(StageArgs A) {
    using T = TriS<N, MAT>;
    using H = P16<PREC>;
    typedef typename H::T h16;
    typedef typename H::V hv;
    constexpr int Np = T::Np, Nfp = T::Nfp, Nafp = T::Nafp, Kd = T::Kd, KS = T::KS, MT = T::MT;
    constexpr int G = T::G, FG = T::FG, RP = T::RP, SUB = T::SUB, BUF = T::BUF, QW = T::QW, JW = T::JW;
    __shared__ float sbuf[2 * BUF];
    __shared__ uint4 sa[2 * MT * KS * 64];  // A fragments: hi then lo, 8 x 16-bit per lane

    const int lane0 = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const bool producer = wv >= 4;
    const int w = wv & 3;

    {
        const uint4 *src = reinterpret_cast<const uint4 *>(A.opsfrag);
        for (int i = threadIdx.x; i < 2 * MT * KS * 64; i += 512) sa[i] = src[i];
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
        float pl[QW];
#pragma unroll
        for (int i = 0; i < QW; ++i) {
            const int r = w + 4 * i;
            pl[i] = r < RP ? qt[(unsigned)(r * 64 + ln)] : 0.f;
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
#pragma unroll
        for (int i = 0; i < QW; ++i) {
            const int r = w + 4 * i;
            if (r < RP) Bp[r * 16] = pl[i];
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

    int it = 0;
    for (int tl = bi; tl < xcount; tl += GB, ++it) {
        const int cur = it & 1;
        if (producer) {
            const int tn = tl + GB;
            if (tn < xcount) {
                produce(xbase + tn, cur ^ 1);
                if (tn + GB < xcount) load_recs(xbase + tn + GB);
            }
        } else {
            const int tile = xbase + tl;
            int lane = lane0;
            asm volatile("" : "+v"(lane));
            const int g = lane >> 4, c = lane & 15;
            const int col = 16 * w + c;
            float *B = sbuf + cur * BUF + w * SUB + c;
            float *rt = A.res + (size_t)tile * (3 * Np * 64);
            float *ot = A.qout + (size_t)tile * (3 * Np * 64);

            float rr[3][MT][4];
#pragma unroll
            for (int f = 0; f < 3; ++f)
#pragma unroll
                for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                    for (int jj = 0; jj < 4; ++jj) {
                        const int n = 16 * mt + 4 * g + jj;
                        rr[f][mt][jj] = n < Np ? rt[(unsigned)((f * Np + n) * 64 + col)] : 0.f;
                    }
            // FP64 geometric factors and face data of column col
            const double *gt = A.geo64 + (size_t)tile * (G * 64);
            const double rx = gt[0 * 64 + col], ry = gt[1 * 64 + col], sx = gt[2 * 64 + col], sy = gt[3 * 64 + col];
            double ieps = 1.0, imu = 1.0;
            if (MAT) {
                ieps = gt[(4 % G) * 64 + col];
                imu = gt[(5 % G) * 64 + col];
            }
            const double *ft = A.fgeo64 + (size_t)tile * (3 * FG * 64);
            double fd[3][FG];
#pragma unroll
            for (int f = 0; f < 3; ++f)
#pragma unroll
                for (int q = 0; q < FG; ++q) fd[f][q] = ft[(f * FG + q) * 64 + col];

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

            // split-precision contraction: K-steps of 32, lane group g holds
            // rows 32 ks + 8 g + q, q = 0..7.  Dr and Ds annihilate constants,
            // so the volume operand is formed from q - q(c) with c a node near
            // the centroid: the split then represents the (small, for resolved
            // fields) variation across the element instead of the field itself.
            constexpr int CN = T::lat(N / 3, N / 3);
            const float hx0 = B[(0 * Np + CN) * 16], hy0 = B[(1 * Np + CN) * 16], ez0 = B[(2 * Np + CN) * 16];
            const double rxH = rx * imu, ryH = ry * imu, sxH = sx * imu, syH = sy * imu;
            const double rxE = rx * ieps, ryE = ry * ieps, sxE = sx * ieps, syE = sy * ieps;
            // FP16 (5-bit exponent) needs a per-element power-of-two scale:
            // the operand column is scaled so that its largest entry is below
            // 2^14 (no overflow of the hi part, lo parts kept out of the
            // subnormal range for entries near the maximum), the result is
            // scaled back exactly.  The bound: volume entries are at most
            // 2 max|g| max|q - q_c|, flux entries are read as they are.
            float scale = 1.f, unscale = 1.f;
            if constexpr (PREC == 2) {
                float mq = 0.f, mf = 0.f;
#pragma unroll
                for (int nb = 0; nb < (Np + 3) / 4; ++nb) {
                    const int n = 4 * nb + g;
                    if (n < Np) {
                        mq = fmaxf(mq, fabsf(B[(0 * Np + n) * 16] - hx0));
                        mq = fmaxf(mq, fabsf(B[(1 * Np + n) * 16] - hy0));
                        mq = fmaxf(mq, fabsf(B[(2 * Np + n) * 16] - ez0));
                    }
                }
#pragma unroll
                for (int jb = 0; jb < (Nafp + 3) / 4; ++jb) {
                    const int j = 4 * jb + g;
                    if (j < Nafp) {
#pragma unroll
                        for (int f = 0; f < 3; ++f) mf = fmaxf(mf, fabsf(B[(RP + f * Nafp + j) * 16]));
                    }
                }
                const double gmax = fmax(fmax(fabs(rx), fabs(ry)), fmax(fabs(sx), fabs(sy))) * fmax(ieps, imu);
                float mx = fmaxf((float)(2.0 * gmax * (double)mq) * 1.0001f, mf);
                mx = fmaxf(mx, __shfl_xor(mx, 16));
                mx = fmaxf(mx, __shfl_xor(mx, 32));
                if (mx > 0.f && mx < 3.0e38f) {
                    int ex;
                    frexpf(mx, &ex);  // mx < 2^ex
                    const int e = 14 - ex;
                    scale = ldexpf(1.f, e);
                    unscale = ldexpf(1.f, -e);
                }
            }
            floatx4 acc[3][MT];
#pragma unroll
            for (int f = 0; f < 3; ++f)
#pragma unroll
                for (int mt = 0; mt < MT; ++mt) acc[f][mt] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int ks = 0; ks < KS; ++ks) {
                hv bh[3], bl[3];
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    // kmin/kmax bound k over the four lane groups at compile
                    // time, so only straddling K-steps select per lane
                    const int kmin = 32 * ks + q, kmax = kmin + 24;
                    const int k = kmin + 8 * g;
                    const bool vol = kmax < 2 * Np ? true : (kmin >= 2 * Np ? false : k < 2 * Np);
                    float val[3];
                    if (vol) {
                        const bool isr = kmax < Np ? true : (kmin >= Np ? false : k < Np);
                        const int node = isr ? k : k - Np;
                        const double hx = B[(0 * Np + node) * 16] - hx0, hy = B[(1 * Np + node) * 16] - hy0;
                        const double ez = B[(2 * Np + node) * 16] - ez0;
                        const double uH = isr ? rxH : sxH, vH = isr ? ryH : syH;
                        const double uE = isr ? rxE : sxE, vE = isr ? ryE : syE;
                        val[0] = (float)(-vH * ez) * scale;
                        val[1] = (float)(uH * ez) * scale;
                        val[2] = (float)(uE * hy - vE * hx) * scale;
                    } else if (k < Kd) {
                        const int jf = k - 2 * Np;
#pragma unroll
                        for (int f = 0; f < 3; ++f) val[f] = B[(RP + f * Nafp + jf) * 16] * scale;
                    } else {
                        val[0] = val[1] = val[2] = 0.f;
                    }
#pragma unroll
                    for (int f = 0; f < 3; ++f) {
                        const h16 hi = (h16)val[f];
                        bh[f][q] = hi;
                        bl[f][q] = (h16)(val[f] - (float)hi);
                    }
                }
#pragma unroll
                for (int mt = 0; mt < MT; ++mt) {
                    const uint4 ahu = sa[(mt * KS + ks) * 64 + lane];
                    const uint4 alu = sa[MT * KS * 64 + (mt * KS + ks) * 64 + lane];
                    hv ah, al;
                    __builtin_memcpy(&ah, &ahu, 16);
                    __builtin_memcpy(&al, &alu, 16);
#pragma unroll
                    for (int f = 0; f < 3; ++f) {
                        acc[f][mt] = H::mfma(ah, bh[f], acc[f][mt]);
                        acc[f][mt] = H::mfma(ah, bl[f], acc[f][mt]);
                        acc[f][mt] = H::mfma(al, bh[f], acc[f][mt]);
                    }
                }
                __builtin_amdgcn_sched_barrier(0);
            }

            // fused low-storage RK update
#pragma unroll
            for (int f = 0; f < 3; ++f)
#pragma unroll
                for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                    for (int jj = 0; jj < 4; ++jj) {
                        const int n = 16 * mt + 4 * g + jj;
                        if (n < Np) {
                            const unsigned idx = (unsigned)((f * Np + n) * 64 + col);
                            const float r = A.a * rr[f][mt][jj] + A.dt * (acc[f][mt][jj] * unscale);
                            rt[idx] = r;
                            ot[idx] = B[(f * Np + n) * 16] + A.b * r;
                        }
                    }
        }
        __syncthreads();
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

// out: 2*MT*KS*64 uint4 (hi fragments, then lo fragments); fragment (mt, ks)
// of lane l holds Op[16 mt + l%16][32 ks + 8 (l/16) + q], q = 0..7.
int opsfrag_split(int dim, int N, int prec, const double *ops_fused, int Kd, void *out) {
    const int Np = dim == 2 ? (N + 1) * (N + 2) / 2 : (N + 1) * (N + 2) * (N + 3) / 6;
    const int KS = (Kd + 31) / 32, MT = (Np + 15) / 16;
    const int n = 2 * MT * KS * 64;
    if (!out) return n * 16;
    uint16_t *o = static_cast<uint16_t *>(out);
    for (int mt = 0; mt < MT; ++mt)
        for (int ks = 0; ks < KS; ++ks)
            for (int l = 0; l < 64; ++l)
                for (int q = 0; q < 8; ++q) {
                    const int row = 16 * mt + (l % 16), k = 32 * ks + 8 * (l / 16) + q;
                    const double v = (row < Np && k < Kd) ? ops_fused[(size_t)row * Kd + k] : 0.0;
                    uint16_t hi, lo;
                    if (prec == 1) {
                        hi = to_bf16_bits((float)v);
                        lo = to_bf16_bits((float)(v - (double)from_bf16_bits(hi)));
                    } else {
                        hi = to_f16_bits((float)v);
                        lo = to_f16_bits((float)(v - (double)from_f16_bits(hi)));
                    }
                    const size_t base = ((size_t)(mt * KS + ks) * 64 + l) * 8 + q;
                    o[base] = hi;
                    o[(size_t)MT * KS * 64 * 8 + base] = lo;
                }
    return n * 16;
}

}  // namespace dgw
