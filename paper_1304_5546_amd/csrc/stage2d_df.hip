// Fused LSRK stage for 2D TM Maxwell, derivative-first, with the
// element-local contractions on the matrix cores of gfx950, in one of two
// arithmetics:
//   R = double: the double-precision variant (fields, residual, operators,
//               factors and every operation in FP64), v_mfma_f64_16x16x4_f64;
//   R = float : FP32 fields and arithmetic, v_mfma_f32_16x16x4_f32.
//
// Derivative-first: for each field u the reference derivatives Dr u and
// Ds u (eq. dg-diff-local-to-global) are two contractions on the matrix
// cores, the chain rule and the curl of eq. dg-strong-explicit act on the
// accumulators, and the LIFT of the three flux components (eq. dg-lift)
// accumulates on top:
//   rhs_Hx = -(r_y Dr Ez + s_y Ds Ez) / mu + LIFT flux_Hx
//   rhs_Hy =  (r_x Dr Ez + s_x Ds Ez) / mu + LIFT flux_Hy
//   rhs_Ez =  (r_x Dr Hy + s_x Ds Hy - r_y Dr Hx - s_y Ds Hx) / eps + LIFT flux_Ez
// with the upwind flux of eq. max2d-numflux (factor 1/2, [q] = q^- - q^+,
// PEC mirror state E+ = -E-, H+ = H- on the wall, exact Riemann flux across
// eps/mu jumps with the material factors folded into its coefficients).
//
// Work unit = one wave and 16 consecutive elements (one MFMA N-tile; lane
// (g, c) = (lane / 16, lane % 16) works on element column c; A fragments hold
// A[16 mt + c][4 ks + g], B fragments B[4 ks + g][c]; value jj of the 16x16
// result holds row 4 g + jj of column c in FP32, row g + 4 jj in FP64).  The B
// fragment of K-step ks is rows 4 ks + g of a field, read straight from
// memory with buffer loads; as they arrive the values are also written to
// the wave's LDS copy of its elements' fields, from which the own face
// traces and the RK update read them.  The flux of face node j = 4 ks + g
// is evaluated in the lane that feeds it to the LIFT contraction as its B
// value, so the flux never goes through memory.  Partner traces are
// gathered through the compressed face record (partner element, face,
// orientation) and the partner-node table.  Waves share only the operator
// fragments and node tables in LDS, so the persistent loop needs no barrier;
// each XCD walks a contiguous range of work units.
#include <hip/hip_runtime.h>

#include "device.hpp"

namespace dgw {

typedef double doublex4 __attribute__((ext_vector_type(4)));
typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

namespace {

// The arithmetic type's product, result-row order, memory access and the
// solve's buffers and coefficients in that type.
template <typename R>
struct Arith;

template <>
struct Arith<double> {
    using V4 = doublex4;
    static constexpr int RG = 1, RJ = 4;  // value jj of lane group g: row RG g + RJ jj
    __device__ static V4 mfma(double a, double b, V4 c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
    __device__ static double load(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
        return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
    }
    __device__ static void store(__amdgpu_buffer_rsrc_t r, double v, unsigned voff, unsigned soff) {
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, voff, soff, 0);
    }
    __host__ __device__ static const double *qin(const StageArgs &A) { return A.qin64; }
    __host__ __device__ static double *qout(const StageArgs &A) { return A.qout64; }
    __host__ __device__ static double *res(const StageArgs &A) { return A.res64; }
    __host__ __device__ static const double *geo(const StageArgs &A) { return A.geo64; }
    __host__ __device__ static const double *fgeo(const StageArgs &A) { return A.fgeo64; }
    __host__ __device__ static const double *frag(const StageArgs &A) { return A.opsfrag64; }
    __device__ static double a(const StageArgs &A) { return A.a64; }
    __device__ static double b(const StageArgs &A) { return A.b64; }
    __device__ static double dt(const StageArgs &A) { return A.dt64; }
    __device__ static double alpha(const StageArgs &A) { return A.alpha64; }
};

template <>
struct Arith<float> {
    using V4 = floatx4;
    static constexpr int RG = 4, RJ = 1;
    __device__ static V4 mfma(float a, float b, V4 c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
    __device__ static float load(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
        return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
    }
    __device__ static void store(__amdgpu_buffer_rsrc_t r, float v, unsigned voff, unsigned soff) {
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, voff, soff, 0);
    }
    __host__ __device__ static const float *qin(const StageArgs &A) { return A.qin; }
    __host__ __device__ static float *qout(const StageArgs &A) { return A.qout; }
    __host__ __device__ static float *res(const StageArgs &A) { return A.res; }
    __host__ __device__ static const float *geo(const StageArgs &A) { return A.geo; }
    __host__ __device__ static const float *fgeo(const StageArgs &A) { return A.fgeo; }
    __host__ __device__ static const float *frag(const StageArgs &A) { return A.opsfrag; }
    __device__ static float a(const StageArgs &A) { return A.a; }
    __device__ static float b(const StageArgs &A) { return A.b; }
    __device__ static float dt(const StageArgs &A) { return A.dt; }
    __device__ static float alpha(const StageArgs &A) { return A.alpha; }
};

// P elements per lane (P = 2: lane c of an MFMA N-tile pair works on
// elements 2 c and 2 c + 1, read and written as one 8-byte access).
template <typename R, int N, bool MAT, int P>
struct TriD {
    static constexpr int Np = (N + 1) * (N + 2) / 2;
    static constexpr int Nfp = N + 1;
    static constexpr int Nafp = 3 * Nfp;
    static constexpr int MT = (Np + 15) / 16;    // M-tiles of the output nodes
    static constexpr int KV = (Np + 3) / 4;      // K-steps of a derivative
    static constexpr int KL = (Nafp + 3) / 4;    // K-steps of LIFT
    static constexpr int AV = 2 * MT * KV * 64;  // Dr, Ds fragments
    static constexpr int AL = MT * KL * 64;      // LIFT fragments
    static constexpr int NT = Nafp + 3 * 2 * Nfp;  // own face nodes, partner-node table
    static constexpr int G = MAT ? 6 : 4;        // per-element factor rows
    static constexpr int FG = MAT ? 6 : 3;       // per-face data rows
    static constexpr int FS = 16 * P + 1;        // LDS row stride of the field copies
    static constexpr int FW = 3 * Np * FS;       // values of one wave's field copy
    // waves per work-group: as many as the LDS holds (field copies plus one
    // shared copy of the operators), at most WMAX: 12 (3 per SIMD, which
    // leaves each wave the ~170 registers that FP64 from order 5, FP32 from
    // order 7 and FP32 element pairs need), else 16
    static constexpr int LDS_MAX = 160 * 1024;
    static constexpr int WMAX = (sizeof(R) == 8 || N >= 7 || P == 2) ? 12 : 16;
    static constexpr int FIXED = (AV + AL) * (int)sizeof(R) + NT * 4;
    // FP32 single-element lanes at order 5: the update goes through a second
    // per-wave buffer and moves 16 bytes per lane
    static constexpr bool TU = sizeof(R) == 4 && P == 1 && N == 5;
    static constexpr int WPB0 = (LDS_MAX - FIXED) / ((TU ? 2 : 1) * FW * (int)sizeof(R));
    static constexpr int WPB = WPB0 >= WMAX ? WMAX : (WPB0 >= 12 ? 12 : (WPB0 >= 8 ? 8 : 4));
};

// Buffer resource over `bytes` bytes at a wave-uniform base: loads past the
// resource's size read 0, stores past it are dropped.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc(const void *p, unsigned bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, (int)bytes, 0x00020000);
}

// P consecutive values of a row (one access), returned by value
template <typename R, int P>
struct PV {
    R v[P];
};
template <typename R, int P>
__device__ __forceinline__ PV<R, P> loadp(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
    PV<R, P> out;
    if constexpr (P == 1) {
        out.v[0] = Arith<R>::load(r, voff, soff);
    } else {
        static_assert(sizeof(R) == 4 && P == 2, "element pairs are FP32 only");
        // through a 64-bit integer: extracting the elements of the two-dword
        // result directly gets the load narrowed to its first dword by this
        // compiler (both elements then read the same value)
        const unsigned long long u =
            __builtin_bit_cast(unsigned long long, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
        out.v[0] = __builtin_bit_cast(R, (unsigned)u);
        out.v[1] = __builtin_bit_cast(R, (unsigned)(u >> 32));
    }
    return out;
}
template <int P>
__device__ __forceinline__ PV<int, P> loadp_i(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
    PV<int, P> out;
    if constexpr (P == 1) {
        out.v[0] = __builtin_bit_cast(int, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
    } else {
        const unsigned long long u =
            __builtin_bit_cast(unsigned long long, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
        out.v[0] = (int)(unsigned)u;
        out.v[1] = (int)(unsigned)(u >> 32);
    }
    return out;
}
template <typename R, int P>
__device__ __forceinline__ void storep(__amdgpu_buffer_rsrc_t r, PV<R, P> x, unsigned voff, unsigned soff) {
    if constexpr (P == 1) {
        Arith<R>::store(r, x.v[0], voff, soff);
    } else {
        const u32x2 u = {__builtin_bit_cast(unsigned, x.v[0]), __builtin_bit_cast(unsigned, x.v[1])};
        __builtin_amdgcn_raw_buffer_store_b64(u, r, voff, soff, 0);
    }
}

// Buffers of the solve and its tile t.
template <typename R>
struct DfSrc {
    const R *qin;
    R *qout, *res;
    const R *geo, *fgeo;
    const int *nbr;
    int tile;
    R dt;
};
template <typename R>
__device__ __forceinline__ DfSrc<R> df_src(const StageArgs &A, int t) {
    using X = Arith<R>;
    return DfSrc<R>{X::qin(A), X::qout(A), X::res(A), X::geo(A), X::fgeo(A), A.nbr, t, X::dt(A)};
}

}  // namespace

// Tuning: K-steps of face traces kept in flight; fields whose residual rows
// are loaded before the surface loop.
#ifndef DGW_DF_SPD
#define DGW_DF_SPD 2
#endif
#ifndef DGW_DF_RPF
#define DGW_DF_RPF 1
#endif

template <typename R, int N, bool MAT, int P>
__global__ void __launch_bounds__((64 * TriD<R, N, MAT, P>::WPB)) stage2d_df_kernel(StageArgs A) {
    using T = TriD<R, N, MAT, P>;
    using X = Arith<R>;
    using V4 = typename X::V4;
    constexpr unsigned W = sizeof(R);  // bytes per value
    constexpr unsigned ROW = 64 * W;   // bytes per tile row
    constexpr int Np = T::Np, Nfp = T::Nfp, Nafp = T::Nafp, MT = T::MT, KV = T::KV, KL = T::KL;
    constexpr int AV = T::AV, AL = T::AL, NT = T::NT, G = T::G, FG = T::FG, FS = T::FS, WPB = T::WPB;
    constexpr int UPT = 4 / P;  // work units per 64-element tile
    __shared__ R sA[AV + AL];
    __shared__ int stab[NT];
    __shared__ R sF[WPB][T::FW];
    __shared__ R sT[T::TU ? WPB : 1][T::TU ? T::FW : 1];  // right-hand side, for the update

    for (int i = threadIdx.x; i < AV + AL; i += 64 * WPB) sA[i] = X::frag(A)[i];
    for (int i = threadIdx.x; i < NT; i += 64 * WPB) stab[i] = A.itab[i];
    __syncthreads();

    const int lane0 = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    R *F = sF[w];

    // work units (16 P elements of a tile) of this XCD: a contiguous range,
    // dealt round-robin to its waves
    const int nunits = UPT * A.ntiles;
    const int x = blockIdx.x & 7, bi = blockIdx.x >> 3, GB = gridDim.x >> 3;
    const int q8 = nunits >> 3, r8 = nunits & 7;
    const int xbase = x * q8 + (x < r8 ? x : r8), xcount = q8 + (x < r8 ? 1 : 0);
    const R hs_alpha = R(0.5) * X::alpha(A);
    constexpr unsigned TB = 3 * Np * ROW;  // bytes of a tile's fields

    for (int ul = bi * WPB + w; ul < xcount; ul += GB * WPB) {
        const int unit = xbase + ul;
        const DfSrc<R> S = df_src<R>(A, unit / UPT);
        const int tile = S.tile;  // tile within the solve
        // lane indices opaque to the compiler, recomputed per work unit
        int lane = lane0;
        asm volatile("" : "+v"(lane));
        const int g = lane >> 4, c = lane & 15;
        const int col = 16 * P * (unit % UPT) + P * c;       // the lane's first element in the tile
        const unsigned vcol = (unsigned)col * W;             // column within a row
        const unsigned vrow = (unsigned)(g * 64 + col) * W;  // row 4 ks + g of a K-step
        const __amdgpu_buffer_rsrc_t rq = rsrc(S.qin + (size_t)tile * (3 * Np * 64), TB);

        R gf[G][P];
        {
            const __amdgpu_buffer_rsrc_t rg = rsrc(S.geo + (size_t)tile * (G * 64), G * ROW);
#pragma unroll
            for (int q = 0; q < G; ++q) {
                const PV<R, P> t = loadp<R, P>(rg, vcol, q * ROW);
#pragma unroll
                for (int p = 0; p < P; ++p) gf[q][p] = t.v[p];
            }
        }
        // face records and face data of the elements, held as scalars
        const __amdgpu_buffer_rsrc_t rn = rsrc(S.nbr + (size_t)tile * (3 * 64), 3 * 64 * 4);
        const __amdgpu_buffer_rsrc_t rf = rsrc(S.fgeo + (size_t)tile * (3 * FG * 64), 3 * FG * ROW);
        const unsigned vcol4 = (unsigned)col * 4;
        int rc[3][P];
#pragma unroll
        for (int f = 0; f < 3; ++f) {
            const PV<int, P> t = loadp_i<P>(rn, vcol4, f * 256);
#pragma unroll
            for (int p = 0; p < P; ++p) rc[f][p] = t.v[p];
        }
        R fd[3 * FG][P];
#pragma unroll
        for (int q = 0; q < 3 * FG; ++q) {
            const PV<R, P> t = loadp<R, P>(rf, vcol, q * ROW);
#pragma unroll
            for (int p = 0; p < P; ++p) fd[q][p] = t.v[p];
        }

        // ---- volume: derivatives of each field, chain rule and curl into cv
        R cv[3][MT][4][P];
#pragma unroll
        for (int f = 0; f < 3; ++f)
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                for (int jj = 0; jj < 4; ++jj)
#pragma unroll
                    for (int p = 0; p < P; ++p) cv[f][mt][jj][p] = R(0);
        // operands of the next field in flight; rows past Np belong to the
        // next field (or lie past the tile, read as 0) and meet zero
        // operator columns
        PV<R, P> bn[KV];
#pragma unroll
        for (int ks = 0; ks < KV; ++ks) bn[ks] = loadp<R, P>(rq, vrow, (4 * ks) * ROW);
#pragma unroll
        for (int f = 0; f < 3; ++f) {
            R bq[KV][P];
#pragma unroll
            for (int ks = 0; ks < KV; ++ks)
#pragma unroll
                for (int p = 0; p < P; ++p) {
                    bq[ks][p] = bn[ks].v[p];
                    if (4 * ks + g < Np) F[(f * Np + 4 * ks + g) * FS + P * c + p] = bq[ks][p];
                }
            if (f + 1 < 3) {
#pragma unroll
                for (int ks = 0; ks < KV; ++ks) bn[ks] = loadp<R, P>(rq, vrow, ((f + 1) * Np + 4 * ks) * ROW);
            }
            V4 d[P][2][MT];
#pragma unroll
            for (int p = 0; p < P; ++p)
#pragma unroll
                for (int o = 0; o < 2; ++o)
#pragma unroll
                    for (int mt = 0; mt < MT; ++mt) d[p][o][mt] = V4{R(0), R(0), R(0), R(0)};
            int la = lane;
            asm volatile("" : "+v"(la));
#pragma unroll
            for (int ks = 0; ks < KV; ++ks)
#pragma unroll
                for (int o = 0; o < 2; ++o)
#pragma unroll
                    for (int mt = 0; mt < MT; ++mt) {
                        const R a = sA[((o * MT + mt) * KV + ks) * 64 + la];
#pragma unroll
                        for (int p = 0; p < P; ++p) d[p][o][mt] = X::mfma(a, bq[ks][p], d[p][o][mt]);
                    }
            // d_x u = r_x Dr u + s_x Ds u, d_y u = r_y Dr u + s_y Ds u
#pragma unroll
            for (int p = 0; p < P; ++p)
#pragma unroll
                for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                    for (int jj = 0; jj < 4; ++jj) {
                        const R dr = d[p][0][mt][jj], ds = d[p][1][mt][jj];
                        const R gx = gf[0][p] * dr + gf[2][p] * ds;
                        const R gy = gf[1][p] * dr + gf[3][p] * ds;
                        if (f == 0) cv[2][mt][jj][p] -= gy;  // Ez: -d_y Hx
                        if (f == 1) cv[2][mt][jj][p] += gx;  // Ez: +d_x Hy
                        if (f == 2) {
                            cv[0][mt][jj][p] -= gy;  // Hx: -d_y Ez
                            cv[1][mt][jj][p] += gx;  // Hy: +d_x Ez
                        }
                    }
#pragma unroll
            for (int o = 0; o < 3; ++o)
#pragma unroll
                for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                    for (int jj = 0; jj < 4; ++jj)
#pragma unroll
                        for (int p = 0; p < P; ++p) asm volatile("" : "+v"(cv[o][mt][jj][p]));
            __builtin_amdgcn_sched_barrier(0);
        }

        // the LIFT contraction accumulates on top of the volume part
        V4 acc[P][3][MT];
#pragma unroll
        for (int p = 0; p < P; ++p)
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) {
                const R im = MAT ? gf[5][p] : R(1), ie = MAT ? gf[4][p] : R(1);
                acc[p][0][mt] = V4{cv[0][mt][0][p] * im, cv[0][mt][1][p] * im, cv[0][mt][2][p] * im, cv[0][mt][3][p] * im};
                acc[p][1][mt] = V4{cv[1][mt][0][p] * im, cv[1][mt][1][p] * im, cv[1][mt][2][p] * im, cv[1][mt][3][p] * im};
                acc[p][2][mt] = V4{cv[2][mt][0][p] * ie, cv[2][mt][1][p] * ie, cv[2][mt][2][p] * ie, cv[2][mt][3][p] * ie};
            }

        // residual rows of the first RPF fields, issued before the surface
        // loop so that their latency overlaps it (pinned there by the
        // scheduling barrier)
        constexpr int RPF = DGW_DF_RPF;
        constexpr int RG = X::RG, RJ = X::RJ;
        const __amdgpu_buffer_rsrc_t rr = rsrc(S.res + (size_t)tile * (3 * Np * 64), TB);
        const unsigned vout = (unsigned)(RG * g * 64 + col) * W;  // row RG g of column col
        PV<R, P> rpre[RPF > 0 && !T::TU ? RPF : 1][MT][4];
        // TU: lane (r0t, qdt) = (lane / 4, lane % 4) owns columns 4 qdt ..
        // 4 qdt + 3 of the unit's 16 in rows r0t + 16 i of the tile; the
        // row is in the per-lane offset, the 16-row step in the (uniform)
        // scalar offset.  The first RPT row groups are loaded here.
        constexpr int NRT = 3 * Np, NIT = (NRT + 15) / 16, RPT = NIT < 2 ? NIT : 2;
        const int r0t = lane >> 2, qdt = lane & 3;
        const unsigned vq = (unsigned)(16 * (unit % UPT) + 4 * qdt) * 4 + (unsigned)r0t * ROW;
        unsigned __int128 rpt[RPT];
        if constexpr (T::TU) {
#pragma unroll
            for (int i = 0; i < RPT; ++i)
                rpt[i] = r0t + 16 * i < NRT
                             ? __builtin_bit_cast(unsigned __int128,
                                                  __builtin_amdgcn_raw_buffer_load_b128(rr, vq, (unsigned)(16 * i) * ROW, 0))
                             : (unsigned __int128)0;
        } else {
#pragma unroll
            for (int f = 0; f < RPF; ++f)
#pragma unroll
                for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                    for (int jj = 0; jj < 4; ++jj)
                        rpre[f][mt][jj] = loadp<R, P>(rr, vout, (f * Np + 16 * mt + RJ * jj) * ROW);
        }
        __builtin_amdgcn_sched_barrier(0);

        // ---- surface: flux at face node j = 4 ks + g, then LIFT
        // The four face nodes 4 ks .. 4 ks + 3 of a K-step lie on at most two
        // faces, lo and hi (fixed once the loop over ks is unrolled): a
        // two-way select per value, with constant array indices (a select
        // over all three faces becomes an indexed scratch-memory lookup).
        auto face_lo = [](int ks) { return (4 * ks < Nafp ? 4 * ks : Nafp - 1) / Nfp; };
        auto face_hi = [](int ks) { return (4 * ks + 3 < Nafp ? 4 * ks + 3 : Nafp - 1) / Nfp; };
        auto face_rec = [&](int ks, bool hi, int p) { return hi ? rc[face_hi(ks)][p] : rc[face_lo(ks)][p]; };
        auto face_val = [&](int ks, bool hi, int q, int p) {
            return hi ? fd[face_hi(ks) * FG + q][p] : fd[face_lo(ks) * FG + q][p];
        };
        // own and partner traces of face node j for element p of the lane
        // (on the wall the partner is the element itself; the mirror sign is
        // applied with the jump)
        auto load_traces = [&](int ks, R (&m)[3][P], R (&pv)[3][P], int (&wall)[P]) {
            const int j = 4 * ks + g;
            const int jc = j < Nafp ? j : Nafp - 1;  // lanes past the faces read a valid node
            const int face = jc / Nfp, i = jc - face * Nfp;
            const bool hi = face > face_lo(ks);
            const int own = stab[jc];
#pragma unroll
            for (int p = 0; p < P; ++p) {
                const int rcv = face_rec(ks, hi, p);
                wall[p] = rcv < 0;
                const int e2 = wall[p] ? tile * 64 + col + p : (rcv >> 5);
                const int pn = wall[p] ? own : stab[Nafp + (((rcv >> 3) & 3) * 2 + (rcv & 7)) * Nfp + i];
                const R *qp = S.qin + tix(e2, pn, 3 * Np);
#pragma unroll
                for (int f = 0; f < 3; ++f) m[f][p] = F[(f * Np + own) * FS + P * c + p];
#pragma unroll
                for (int f = 0; f < 3; ++f) pv[f][p] = qp[(size_t)f * Np * 64];
            }
        };
        constexpr int SPD = DGW_DF_SPD;  // K-steps of traces in flight
        R mb[SPD][3][P], pb[SPD][3][P];
        int wb[SPD][P];
#pragma unroll
        for (int s0 = 0; s0 < SPD; ++s0)
            if (s0 < KL) load_traces(s0, mb[s0], pb[s0], wb[s0]);
#pragma unroll
        for (int ks = 0; ks < KL; ++ks) {
            R m[3][P], pv[3][P];
            int wall[P];
            const int slot = ks % SPD;
#pragma unroll
            for (int p = 0; p < P; ++p) {
                wall[p] = wb[slot][p];
#pragma unroll
                for (int f = 0; f < 3; ++f) {
                    m[f][p] = mb[slot][f][p];
                    pv[f][p] = pb[slot][f][p];
                }
            }
            if (ks + SPD < KL) load_traces(ks + SPD, mb[slot], pb[slot], wb[slot]);
            const int j = 4 * ks + g;
            const bool hi = (j < Nafp ? j : Nafp - 1) / Nfp > face_lo(ks);
            const R on = j < Nafp ? R(1) : R(0);  // lanes past the faces feed zero rows
            R fl[3][P];
#pragma unroll
            for (int p = 0; p < P; ++p) {
                // [q] = q- - q+, with q+ = (H-, -E-) on the wall
                const R dHx = m[0][p] - pv[0][p], dHy = m[1][p] - pv[1][p];
                const R dEz = m[2][p] - (wall[p] ? -pv[2][p] : pv[2][p]);
                const R nx = face_val(ks, hi, 0, p), ny = face_val(ks, hi, 1, p);
                const R dh = nx * dHy - ny * dHx;  // jump of the tangential field
                R cEE, cEh, cHE, cHh;
                if (MAT) {
                    cEE = face_val(ks, hi, 2, p);
                    cEh = face_val(ks, hi, 3, p);
                    cHE = face_val(ks, hi, 4, p);
                    cHh = face_val(ks, hi, 5, p);
                } else {
                    const R fs = face_val(ks, hi, 2, p);
                    cEE = hs_alpha * fs;
                    cEh = R(0.5) * fs;
                    cHE = R(0.5) * fs;
                    cHh = hs_alpha * fs;
                }
                const R fE = -(cEE * dEz + cEh * dh) * on;
                const R fH = (cHE * dEz + cHh * dh) * on;
                fl[0][p] = ny * fH;
                fl[1][p] = -nx * fH;
                fl[2][p] = fE;
            }
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) {
                const R a = sA[AV + (mt * KL + ks) * 64 + lane];
#pragma unroll
                for (int p = 0; p < P; ++p)
#pragma unroll
                    for (int f = 0; f < 3; ++f) acc[p][f][mt] = X::mfma(a, fl[f][p], acc[p][f][mt]);
            }
            __builtin_amdgcn_sched_barrier(0);
        }

        // ---- fused low-storage RK update: res <- a res + dt rhs,
        // q_out <- q_in + b res; per field all loads, then the arithmetic,
        // then the stores.  Value jj of M-tile mt is node
        // 16 mt + RG g + RJ jj; rows >= Np are not stored.
        const __amdgpu_buffer_rsrc_t ro = rsrc(S.qout + (size_t)tile * (3 * Np * 64), TB);
        const R ca = X::a(A), cb = X::b(A), cdt = S.dt;
        if constexpr (T::TU) {
            // the right-hand side into the wave's second buffer (node-major,
            // as the field copy), then per lane 4 consecutive columns of a
            // row: one 16-byte load of res, one 16-byte store each of res
            // and q_out
            R *Tb = sT[w];
#pragma unroll
            for (int f = 0; f < 3; ++f)
#pragma unroll
                for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                    for (int jj = 0; jj < 4; ++jj) {
                        const int n = 16 * mt + RG * g + RJ * jj;
                        if (n < Np) Tb[(f * Np + n) * FS + c] = acc[0][f][mt][jj];
                    }
#pragma unroll
            for (int i = 0; i < NIT; ++i) {
                const int r = r0t + 16 * i;
                if (r < NRT) {
                    // through a 128-bit integer: extracting the elements of
                    // the vector result directly gets the load narrowed to
                    // one dword by this compiler
                    const unsigned __int128 ru =
                        i < RPT ? rpt[i < RPT ? i : 0]
                                : __builtin_bit_cast(unsigned __int128, __builtin_amdgcn_raw_buffer_load_b128(
                                                                            rr, vq, (unsigned)(16 * i) * ROW, 0));
                    u32x4 rn, qn;
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        const R rk = ca * __builtin_bit_cast(R, (unsigned)(ru >> (32 * k))) + cdt * Tb[r * FS + 4 * qdt + k];
                        rn[k] = __builtin_bit_cast(unsigned, rk);
                        qn[k] = __builtin_bit_cast(unsigned, F[r * FS + 4 * qdt + k] + cb * rk);
                    }
                    __builtin_amdgcn_raw_buffer_store_b128(rn, rr, vq, (unsigned)(16 * i) * ROW, 0);
                    __builtin_amdgcn_raw_buffer_store_b128(qn, ro, vq, (unsigned)(16 * i) * ROW, 0);
                }
            }
        } else
#pragma unroll
        for (int f = 0; f < 3; ++f) {
            PV<R, P> rv[MT][4], qv[MT][4];
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                for (int jj = 0; jj < 4; ++jj) {
                    const unsigned so = (f * Np + 16 * mt + RJ * jj) * ROW;
                    rv[mt][jj] = f < RPF && !T::TU ? rpre[f < RPF ? f : 0][mt][jj] : loadp<R, P>(rr, vout, so);
                    const int n = 16 * mt + RG * g + RJ * jj;
#pragma unroll
                    for (int p = 0; p < P; ++p) qv[mt][jj].v[p] = n < Np ? F[(f * Np + n) * FS + P * c + p] : R(0);
                }
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                for (int jj = 0; jj < 4; ++jj)
#pragma unroll
                    for (int p = 0; p < P; ++p) {
                        rv[mt][jj].v[p] = ca * rv[mt][jj].v[p] + cdt * acc[p][f][mt][jj];
                        qv[mt][jj].v[p] = qv[mt][jj].v[p] + cb * rv[mt][jj].v[p];
                    }
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                for (int jj = 0; jj < 4; ++jj) {
                    if (16 * mt + RG * g + RJ * jj < Np) {
                        const unsigned so = (f * Np + 16 * mt + RJ * jj) * ROW;
                        storep<R, P>(rr, rv[mt][jj], vout, so);
                        storep<R, P>(ro, qv[mt][jj], vout, so);
                    }
                }
        }
    }
}

namespace {

// P: elements per lane (1, or 2 for the FP32 kernel: element pairs)
template <typename R, int N, bool MAT, int P>
hipError_t launch_df(const StageArgs &a, hipStream_t s) {
    using X = Arith<R>;
    // every pointer the kernel dereferences must be set
    const bool bufs = X::qin(a) && X::qout(a) && X::res(a) && X::geo(a) && X::fgeo(a) && a.nbr;
    if (!X::frag(a) || !a.itab || !bufs || a.ntiles <= 0 || a.ngroups < 8 || (a.ngroups & 7))
        return hipErrorInvalidValue;
    hipLaunchKernelGGL((stage2d_df_kernel<R, N, MAT, P>), dim3(a.ngroups), dim3(64 * TriD<R, N, MAT, P>::WPB), 0, s,
                       a);
    return hipGetLastError();
}

template <typename R, int N, bool MAT, int P>
int occupancy_df() {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, stage2d_df_kernel<R, N, MAT, P>,
                                                     64 * TriD<R, N, MAT, P>::WPB, 0) != hipSuccess)
        return 1;
    return nb > 0 ? nb : 1;
}

template <typename R>
int frag_df(int N, const double *Dr, const double *Ds, const double *LIFT, R *out) {
    const int Np = (N + 1) * (N + 2) / 2, Nafp = 3 * (N + 1);
    const int MT = (Np + 15) / 16, KV = (Np + 3) / 4, KL = (Nafp + 3) / 4;
    const int AV = 2 * MT * KV * 64, AL = MT * KL * 64;
    if (!out) return AV + AL;
    const double *D[2] = {Dr, Ds};
    for (int p = 0; p < 2; ++p)
        for (int mt = 0; mt < MT; ++mt)
            for (int ks = 0; ks < KV; ++ks)
                for (int l = 0; l < 64; ++l) {
                    const int row = 16 * mt + (l % 16), k = 4 * ks + l / 16;
                    out[((p * MT + mt) * KV + ks) * 64 + l] = (row < Np && k < Np) ? (R)D[p][row * Np + k] : R(0);
                }
    for (int mt = 0; mt < MT; ++mt)
        for (int ks = 0; ks < KL; ++ks)
            for (int l = 0; l < 64; ++l) {
                const int row = 16 * mt + (l % 16), k = 4 * ks + l / 16;
                out[AV + (mt * KL + ks) * 64 + l] = (row < Np && k < Nafp) ? (R)LIFT[row * Nafp + k] : R(0);
            }
    return AV + AL;
}

}  // namespace

#define DGW_ORDERS(X) X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8)

hipError_t launch_stage2d_df(int N, bool material, bool fp64, int pairs, const StageArgs &a, hipStream_t s) {
    if (pairs != 1 && (pairs != 2 || fp64)) return hipErrorInvalidValue;
    switch (N) {
#define DGW_CASE(n)                                                                                              \
    case n:                                                                                                      \
        if (fp64) return material ? launch_df<double, n, true, 1>(a, s) : launch_df<double, n, false, 1>(a, s); \
        if (pairs == 2) return material ? launch_df<float, n, true, 2>(a, s) : launch_df<float, n, false, 2>(a, s); \
        return material ? launch_df<float, n, true, 1>(a, s) : launch_df<float, n, false, 1>(a, s);
        DGW_ORDERS(DGW_CASE)
#undef DGW_CASE
        default: return hipErrorInvalidValue;
    }
}

int blocks_per_cu_2d_df(int N, bool material, bool fp64, int pairs) {
    switch (N) {
#define DGW_CASE(n)                                                                                              \
    case n:                                                                                                      \
        if (fp64) return material ? occupancy_df<double, n, true, 1>() : occupancy_df<double, n, false, 1>();   \
        if (pairs == 2) return material ? occupancy_df<float, n, true, 2>() : occupancy_df<float, n, false, 2>(); \
        return material ? occupancy_df<float, n, true, 1>() : occupancy_df<float, n, false, 1>();
        DGW_ORDERS(DGW_CASE)
#undef DGW_CASE
        default: return 1;
    }
}

// A-fragment order of the derivative-first kernel's operators: Dr, Ds
// (out[((p*MT + mt)*KV + ks)*64 + l] = D_p[16 mt + l%16][4 ks + l/16]), then
// LIFT (out[AV + (mt*KL + ks)*64 + l] = LIFT[16 mt + l%16][4 ks + l/16]);
// zero outside the matrices.  Returns the number of values.
int opsfrag2d_df(int N, const double *Dr, const double *Ds, const double *LIFT, float *out) {
    return frag_df<float>(N, Dr, Ds, LIFT, out);
}
int opsfrag2d_df64(int N, const double *Dr, const double *Ds, const double *LIFT, double *out) {
    return frag_df<double>(N, Dr, Ds, LIFT, out);
}

}  // namespace dgw
