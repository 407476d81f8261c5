// Fused LSRK stage for 2D TM Maxwell, FP32, with the element-local
// contractions on the matrix cores (v_mfma_f32_16x16x4_f32) of gfx950.
//
// The right-hand side of eq. dg-strong-explicit is written as ONE contraction
// per output field with the fused operator Op = [Dr | Ds | LIFT]
// (Np x (2 Np + 3 Nfp)): since the geometric factors of an affine element are
// constants, (r_x Dr + s_x Ds) u = Dr (r_x u) + Ds (s_x u), so
//   rhs_Hx = Op [-r_y Ez; -s_y Ez; flux_Hx] / mu
//   rhs_Hy = Op [ r_x Ez;  s_x Ez; flux_Hy] / mu
//   rhs_Ez = Op [r_x Hy - r_y Hx; s_x Hy - s_y Hx; flux_Ez] / eps
// (the material factors of the flux are folded into its coefficients).
//
// Persistent, warp-specialised kernel.  A work-group of 8 waves walks a
// contiguous run of 64-element tiles inside its XCD's share of the mesh:
//   - waves 4..7 (producers) stream tile i+1 into one half of a
//     double-buffered LDS tile: the fields, the geometric factors, the face
//     data and the partner traces of every face node (gathered through the
//     compressed face record: partner element, face, orientation; on the PEC
//     wall the mirror state E+ = -E-, H+ = H- of the element's own trace);
//   - waves 0..3 (consumers) compute tile i from the other half: consumer w
//     owns the MFMA N-tile of elements 16w..16w+15.  It contracts the volume
//     part of K, evaluates the upwind flux (eq. max2d-numflux with the factor
//     1/2, [q] = q^- - q^+, exact Riemann flux across eps/mu jumps) of its own
//     16 elements in place of their partner traces, contracts the flux part of
//     K (the LIFT columns), and applies res <- a res + dt rhs,
//     q_out <- q_in + b res.
// The A fragments of Op stay in LDS for the whole kernel; the B fragments are
// formed on the fly from the LDS tile (times the lane's geometric factors).
// One barrier per tile hands the buffers over.
#include <hip/hip_runtime.h>

#include "device.hpp"

namespace dgw {

typedef float floatx4 __attribute__((ext_vector_type(4)));

// 4x4x1 products for a last M-tile of at most 4 rows (1) or 16x16x4 (0).
#ifndef DGW_MF_TAIL4
#define DGW_MF_TAIL4 1
#endif
// Orders whose last 16-row M-tile holds at most 4 operator rows (with two or
// more M-tiles): those rows are contracted on v_mfma_f32_4x4x1f32 (16 blocks
// of 4x4, a quarter of the 16x16x4 product's matrix-core time).  Block b =
// lane/4 takes K row 4 ks + b/4 and columns 4 (b%4) .. + 3, so the B
// fragment is the 16x16x4 one unchanged; A holds rows 16 (MT-1) + lane%4;
// the four K-partitions are summed across lane groups after the K loops.
constexpr bool tail4_rows(int N) {
    const int Np = (N + 1) * (N + 2) / 2, MT = (Np + 15) / 16;
    return DGW_MF_TAIL4 && MT >= 2 && Np - 16 * (MT - 1) <= 4;
}

namespace {

template <int N, bool MAT>
struct Tri {
    static constexpr int Np = (N + 1) * (N + 2) / 2;
    static constexpr int Nfp = N + 1;
    static constexpr int Nafp = 3 * Nfp;
    static constexpr int Kd = 2 * Np + Nafp;
    static constexpr int KS = (Kd + 3) / 4;
    static constexpr int MT = (Np + 15) / 16;
    // the last M-tile holds at most 4 rows: contracted on 4x4x1 products
    static constexpr bool TAIL4 = tail4_rows(N);
    static constexpr int KV = (2 * Np) / 4;  // K-steps made only of volume columns
    static constexpr int G = MAT ? 6 : 4;    // per-element factor rows
    static constexpr int FG = MAT ? 6 : 3;   // per-face data rows
    // LDS tile rows (each row = 64 elements, stored as 4 sub-tiles of 16)
    static constexpr int RQ = 0;                 // fields f*Np + n
    static constexpr int RG = 3 * Np;            // geometric factors
    static constexpr int RF = RG + G;            // face data face*FG + q
    static constexpr int RP = RF + 3 * FG;       // partner traces / flux f*Nafp + j
    static constexpr int R = RP + 3 * Nafp;
    // sub-tile stride: an odd number of 16-float rows keeps 64-lane row
    // accesses free of bank conflicts
    static constexpr int SUB = R * 16 + ((R & 1) ? 0 : 16);
    static constexpr int BUF = 4 * SUB;
    static constexpr int JW = (Nafp + 3) / 4;    // face nodes per producer wave
    // index of lattice node (i, j) in the order "for j, for i in 0..N-j"
    __host__ __device__ static constexpr int lat(int i, int j) { return j * (N + 1) - j * (j - 1) / 2 + i; }
    // t-th node of face f, faces traversed v0->v1, v1->v2, v2->v0
    __host__ __device__ static constexpr int face_node(int f, int t) {
        return f == 0 ? t : (f == 1 ? lat(N - t, t) : lat(0, N - t));
    }
};

// Buffers of the solve that owns global tile t, and t's index inside it.
struct TileSrc {
    const float *qin;
    float *qout;
    float *res;
    const float *geo, *fgeo;
    const int *nbr;
    int tile;
    float dt;
};

template <bool BATCH>
__device__ __forceinline__ TileSrc tile_src(const StageArgs &A, int t) {
    if constexpr (!BATCH) {
        return TileSrc{A.qin, A.qout, A.res, A.geo, A.fgeo, A.nbr, t, A.dt};
    } else {
        // t is wave-uniform, so these are scalar loads of the descriptor
        const int r = __builtin_amdgcn_readfirstlane(A.tile_req[t]);
        const BatchDesc &d = A.batch[r];
        const int ci = (d.cur0 ^ A.parity) & 1;
        return TileSrc{d.q[ci], d.q[ci ^ 1], d.res, d.geo, d.fgeo, d.nbr, t - d.tile0, d.dt};
    }
}

}  // namespace

// Consumer K-steps between scheduling fences (0: none): the fences keep the
// operand reads of later K-steps from being hoisted into long-lived registers.
#ifndef DGW_MF_SB
#define DGW_MF_SB 2
#endif

// Highest order whose consumers load the residual rows of their next tile at
// the end of the current one.
#ifndef DGW_MF_XRES_MAX
#define DGW_MF_XRES_MAX 6
#endif
// Producer pause (units of 64 cycles) at the top of each tile, so that the
// consumers' residual loads are issued ahead of the producers' stream.
#ifndef DGW_MF_PSLEEP
#define DGW_MF_PSLEEP 0
#endif

template <int N, bool MAT, bool BATCH>
__global__ void __launch_bounds__(512) stage2d_mfma_kernel(StageArgs A) {
    using T = Tri<N, MAT>;
    constexpr int Np = T::Np, Nfp = T::Nfp, Nafp = T::Nafp, Kd = T::Kd, KS = T::KS, MT = T::MT, KV = T::KV;
    constexpr int G = T::G, FG = T::FG, RG = T::RG, RF = T::RF, RP = T::RP, SUB = T::SUB, BUF = T::BUF;
    constexpr int JW = T::JW;
    __shared__ float sbuf[2 * BUF];
    __shared__ float sa[MT * KS * 64];

    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const bool producer = wv >= 4;
    const int w = wv & 3;
    const int g = lane >> 4, c = lane & 15;

    for (int i = threadIdx.x; i < MT * KS * 64; i += 512) sa[i] = A.opsfrag[i];

    // tiles of this XCD: a contiguous range, dealt round-robin to its groups
    const int x = blockIdx.x & 7, bi = blockIdx.x >> 3, GB = gridDim.x >> 3;
    const int q8 = A.ntiles >> 3, r8 = A.ntiles & 7;
    const int xbase = x * q8 + (x < r8 ? x : r8), xcount = q8 + (x < r8 ? 1 : 0);
    if (bi >= xcount) return;  // whole group exits: no tile for it

    // producer state: face records of the next tile to load
    const int prow = (lane >> 4) * SUB + (lane & 15);  // LDS base of element `lane`
    int rec_next[3] = {-1, -1, -1};
    // Addressing: a tile's rows start at a wave-uniform base (kept in scalar
    // registers), the lane adds a small unsigned 32-bit offset row*64 + lane
    // (unsigned, so no 64-bit sign extensions are formed and kept live).
    auto load_recs = [&](int tile) {
        const TileSrc S = tile_src<BATCH>(A, tile);
        const int *nt = S.nbr + (size_t)S.tile * (3 * 64);
        int ln = lane;
        asm volatile("" : "+v"(ln));
#pragma unroll
        for (int f = 0; f < 3; ++f) rec_next[f] = nt[(unsigned)(f * 64 + ln)];
    };
    // stream tile `tile` into buffer `b` (producer waves only)
    auto produce = [&](int tile, int b) {
        const TileSrc S = tile_src<BATCH>(A, tile);
        const float *qt = S.qin + (size_t)S.tile * (3 * Np * 64);
        const float *gt = S.geo + (size_t)S.tile * (G * 64);
        const float *ft = S.fgeo + (size_t)S.tile * (3 * FG * 64);
        int rec[3] = {rec_next[0], rec_next[1], rec_next[2]};
        // lane index opaque to the compiler: keeps the per-row offsets of this
        // role from being hoisted out of the tile loop, where they would stay
        // live (and occupy registers) in the other role's code as well
        int ln = lane;
        asm volatile("" : "+v"(ln));
        // plain rows (fields, factors, face data) in quads of 4 rows x 64
        // elements, one 16-byte access per lane: lane l takes row
        // 4 quad + l/16, elements 4 (l%16) .. 4 (l%16) + 3; producer w
        // takes quads w, w + 4, ...
        constexpr int PV = ((RP + 3) / 4 + 3) / 4;
        floatx4 pv[PV];
        const int lr = ln >> 4, le = 4 * (ln & 15);
#pragma unroll
        for (int i = 0; i < PV; ++i) {
            const int r = 4 * (w + 4 * i) + lr;
            const float *src = r < RG ? qt + r * 64 : (r < RF ? gt + (r - RG) * 64 : ft + (r - RF) * 64);
            pv[i] = r < RP ? *reinterpret_cast<const floatx4 *>(src + le) : floatx4{0.f, 0.f, 0.f, 0.f};
        }
        // partner traces of the face nodes j = w + 4 i
        float pt[JW][3];
#pragma unroll
        for (int i = 0; i < JW; ++i) {
            const int j = w + 4 * i;
            pt[i][0] = pt[i][1] = pt[i][2] = 0.f;
            if (j < Nafp) {
                const int face = j / Nfp, t = j - face * Nfp;
                const int rc = rec[face];
                const bool wall = rc < 0;
                const int e2 = wall ? S.tile * 64 + ln : (rc >> 5);
                const int pn = wall ? T::face_node(face, t) : T::face_node((rc >> 3) & 3, (rc & 7) ? N - t : t);
                // 32-bit element index of (e2, row pn) in the tiled layout
                const unsigned i0 = ((unsigned)(e2 >> 6) * (3 * Np) + pn) * 64 + (e2 & 63);
#pragma unroll
                for (int f = 0; f < 3; ++f) pt[i][f] = S.qin[i0 + f * Np * 64];
                if (wall) pt[i][2] = -pt[i][2];  // PEC mirror: Ez+ = -Ez-, H+ = H-
            }
        }
        float *B = sbuf + b * BUF + prow;
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
                for (int f = 0; f < 3; ++f) B[(RP + f * Nafp + j) * 16] = pt[i][f];
            }
        }
    };

    if (producer) {
        load_recs(xbase + bi);
        produce(xbase + bi, 0);
        if (bi + GB < xcount) load_recs(xbase + bi + GB);
    }
    __syncthreads();

    // Consumer memory traffic is row-major and 16 bytes wide: lane l covers
    // field rows 16 rg + l/4 and, of the wave's 16 elements, the four columns
    // 4 (l%4) .. 4 (l%4) + 3 (one 64-byte run per row).  The residual rows are
    // loaded so; at the end of the tile the right-hand side is transposed to
    // that order through the wave's own LDS sub-tile.  One 16-byte access per
    // row group instead of one 4-byte access per row and lane group keeps
    // the consumers' vector-memory instructions (which queue behind the
    // producers' stream) to 3 RGN per tile.
    constexpr int RGN = (3 * Np + 15) / 16;
    // the residual rows of the next tile are loaded at the end of the current
    // one (in flight across the barrier) up to order DGW_MF_XRES_MAX, else at
    // tile start
    constexpr bool XRES = N <= DGW_MF_XRES_MAX;
    floatx4 rrn[RGN];
    auto load_res = [&](int tile) {
        const TileSrc S = tile_src<BATCH>(A, tile);
        int ln = lane;
        asm volatile("" : "+v"(ln));
        const float *rt = S.res + (size_t)S.tile * (3 * Np * 64) + 16 * w + 4 * (ln & 3);
#pragma unroll
        for (int rg = 0; rg < RGN; ++rg) {
            const int row = 16 * rg + (ln >> 2);
            rrn[rg] = row < 3 * Np ? *reinterpret_cast<const floatx4 *>(rt + (unsigned)(row * 64))
                                   : floatx4{0.f, 0.f, 0.f, 0.f};
        }
    };
    if (XRES && !producer) load_res(xbase + bi);

    // Producer and consumer waves run separate tile loops with the same
    // (wave-uniform) trip count and one barrier per tile each: the barrier
    // counts waves, not program locations.  One loop with a role branch
    // inside would join the roles' register state at the barrier, and the
    // compiler would copy the consumers' in-flight prefetch registers there
    // (waiting for the loads).
    if (producer) {
        int it = 0;
        for (int tl = bi; tl < xcount; tl += GB, ++it) {
            const int cur = it & 1;
            const int tn = tl + GB;
            if (DGW_MF_PSLEEP > 0) __builtin_amdgcn_s_sleep(DGW_MF_PSLEEP);
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
            const TileSrc S = tile_src<BATCH>(A, tile);
            float *rt = S.res + (size_t)S.tile * (3 * Np * 64);
            float *ot = S.qout + (size_t)S.tile * (3 * Np * 64);
            const float dt = S.dt;
            const float *B = sbuf + cur * BUF + w * SUB + c;  // this wave's sub-tile, column c
            float *Bw = sbuf + cur * BUF + w * SUB + c;

            if (!XRES) load_res(tile);
            floatx4 rr[RGN];
#pragma unroll
            for (int rg = 0; rg < RGN; ++rg) rr[rg] = rrn[rg];

            const float rx = B[(RG + 0) * 16], ry = B[(RG + 1) * 16];
            const float sx = B[(RG + 2) * 16], sy = B[(RG + 3) * 16];
            float ieps = 1.f, imu = 1.f;
            if (MAT) {
                ieps = B[(RG + 4 % G) * 16];
                imu = B[(RG + 5 % G) * 16];
            }
            const float rxH = rx * imu, ryH = ry * imu, sxH = sx * imu, syH = sy * imu;
            const float rxE = rx * ieps, ryE = ry * ieps, sxE = sx * ieps, syE = sy * ieps;

            // volume part of K
            floatx4 acc[3][MT];
#pragma unroll
            for (int f = 0; f < 3; ++f)
#pragma unroll
                for (int mt = 0; mt < MT; ++mt) acc[f][mt] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int ks = 0; ks < KV; ++ks) {
                const int k = 4 * ks + g;
                const bool isr = 4 * ks + 3 < Np ? true : (4 * ks >= Np ? false : k < Np);
                const int node = isr ? k : k - Np;
                const float hx = B[(0 * Np + node) * 16];
                const float hy = B[(1 * Np + node) * 16];
                const float ez = B[(2 * Np + node) * 16];
                const float uH = isr ? rxH : sxH, vH = isr ? ryH : syH;
                const float uE = isr ? rxE : sxE, vE = isr ? ryE : syE;
                const float b0 = -vH * ez, b1 = uH * ez, b2 = uE * hy - vE * hx;
#pragma unroll
                for (int mt = 0; mt < MT; ++mt) {
                    const float a = sa[(mt * KS + ks) * 64 + lane];
                    if (T::TAIL4 && mt == MT - 1) {
                        acc[0][mt] = __builtin_amdgcn_mfma_f32_4x4x1f32(a, b0, acc[0][mt], 0, 0, 0);
                        acc[1][mt] = __builtin_amdgcn_mfma_f32_4x4x1f32(a, b1, acc[1][mt], 0, 0, 0);
                        acc[2][mt] = __builtin_amdgcn_mfma_f32_4x4x1f32(a, b2, acc[2][mt], 0, 0, 0);
                    } else {
                        acc[0][mt] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b0, acc[0][mt], 0, 0, 0);
                        acc[1][mt] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b1, acc[1][mt], 0, 0, 0);
                        acc[2][mt] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b2, acc[2][mt], 0, 0, 0);
                    }
                }
                // keep the operand reads of later K-steps from being hoisted
                // into long-lived registers
                if (DGW_MF_SB > 0 && ks % DGW_MF_SB == DGW_MF_SB - 1) __builtin_amdgcn_sched_barrier(0);
            }

            // upwind flux of this wave's 16 elements (lane group g takes face
            // nodes j = g, g+4, ...), written over the partner traces
#pragma unroll
            for (int jb = 0; jb < (Nafp + 3) / 4; ++jb) {
                const int j = 4 * jb + g;
                if (j < Nafp) {
                    const int face = j / Nfp, t = j - face * Nfp;
                    const int own = T::face_node(face, t);
                    const float mHx = B[(0 * Np + own) * 16];
                    const float mHy = B[(1 * Np + own) * 16];
                    const float mEz = B[(2 * Np + own) * 16];
                    const float pHx = B[(RP + 0 * Nafp + j) * 16];
                    const float pHy = B[(RP + 1 * Nafp + j) * 16];
                    const float pEz = B[(RP + 2 * Nafp + j) * 16];
                    const float *fg = B + (RF + face * FG) * 16;
                    const float nx = fg[0], ny = fg[16];
                    const float dHx = mHx - pHx, dHy = mHy - pHy, dEz = mEz - pEz;
                    const float dh = nx * dHy - ny * dHx;
                    float cEE, cEh, cHE, cHh;
                    if (MAT) {
                        cEE = fg[2 * 16];
                        cEh = fg[(3 % FG) * 16];
                        cHE = fg[(4 % FG) * 16];
                        cHh = fg[(5 % FG) * 16];
                    } else {
                        const float hs = 0.5f * fg[2 * 16];
                        cEE = A.alpha * hs;
                        cEh = hs;
                        cHE = hs;
                        cHh = A.alpha * hs;
                    }
                    const float fE = -(cEE * dEz + cEh * dh);
                    const float fH = cHE * dEz + cHh * dh;
                    Bw[(RP + 0 * Nafp + j) * 16] = ny * fH;
                    Bw[(RP + 1 * Nafp + j) * 16] = -nx * fH;
                    Bw[(RP + 2 * Nafp + j) * 16] = fE;
                }
            }

            // flux part of K (including a K-step that straddles the boundary)
#pragma unroll
            for (int ks = KV; ks < KS; ++ks) {
                const int k = 4 * ks + g;
                const bool vol = k < 2 * Np;
                const bool ok = k < Kd;
                const int node = vol ? k - Np : 0;
                const int jc = (!vol && ok) ? k - 2 * Np : 0;
                float b0 = ok ? B[(RP + 0 * Nafp + jc) * 16] : 0.f;
                float b1 = ok ? B[(RP + 1 * Nafp + jc) * 16] : 0.f;
                float b2 = ok ? B[(RP + 2 * Nafp + jc) * 16] : 0.f;
                if (4 * ks < 2 * Np) {  // straddling step: s-part rows for k < 2 Np
                    const float hx = B[(0 * Np + node) * 16];
                    const float hy = B[(1 * Np + node) * 16];
                    const float ez = B[(2 * Np + node) * 16];
                    b0 = vol ? -syH * ez : b0;
                    b1 = vol ? sxH * ez : b1;
                    b2 = vol ? sxE * hy - syE * hx : b2;
                }
#pragma unroll
                for (int mt = 0; mt < MT; ++mt) {
                    const float a = sa[(mt * KS + ks) * 64 + lane];
                    if (T::TAIL4 && mt == MT - 1) {
                        acc[0][mt] = __builtin_amdgcn_mfma_f32_4x4x1f32(a, b0, acc[0][mt], 0, 0, 0);
                        acc[1][mt] = __builtin_amdgcn_mfma_f32_4x4x1f32(a, b1, acc[1][mt], 0, 0, 0);
                        acc[2][mt] = __builtin_amdgcn_mfma_f32_4x4x1f32(a, b2, acc[2][mt], 0, 0, 0);
                    } else {
                        acc[0][mt] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b0, acc[0][mt], 0, 0, 0);
                        acc[1][mt] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b1, acc[1][mt], 0, 0, 0);
                        acc[2][mt] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b2, acc[2][mt], 0, 0, 0);
                    }
                }
                // keep the operand reads of later K-steps from being hoisted
                // into long-lived registers
                if (DGW_MF_SB > 0 && ks % DGW_MF_SB == DGW_MF_SB - 1) __builtin_amdgcn_sched_barrier(0);
            }

            // 4x4x1 tail: sum the four K-partitions (lane groups) of rows
            // 16 (MT-1) + jj; lane group 0 then holds them as the 16x16x4
            // layout would
            if constexpr (T::TAIL4) {
#pragma unroll
                for (int f = 0; f < 3; ++f)
#pragma unroll
                    for (int jj = 0; jj < 4; ++jj) {
                        float v = acc[f][MT - 1][jj];
                        v += __shfl_xor(v, 16);
                        v += __shfl_xor(v, 32);
                        acc[f][MT - 1][jj] = v;
                    }
            }
            // fused low-storage RK update, row-major.  The lane's q_in rows are
            // read first; the right-hand side (rows 16mt+4g+jj of column c in
            // the accumulators) is then written over the sub-tile's field rows
            // and read back in the row-major order (LDS operations of one wave
            // complete in order).
            float *Bs = Bw - c;
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
                        if (n < Np) Bw[(f * Np + n) * 16] = acc[f][mt][jj];
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
                        r[q] = A.a * rr[rg][q] + dt * rh[q];
                        qo[q] = qv[rg][q] + A.b * r[q];
                    }
                    *reinterpret_cast<floatx4 *>(rtl + (unsigned)(row * 64)) = r;
                    *reinterpret_cast<floatx4 *>(otl + (unsigned)(row * 64)) = qo;
                }
            }
            // unconditional (the last tile re-reads its own rows, unused): a
            // conditional prefetch makes the compiler copy the loop-carried
            // registers, waiting for the loads, before the barrier
            if (XRES) load_res(xbase + (tl + GB < xcount ? tl + GB : tl));
            __syncthreads();
        }
    }
}

template <int N, bool MAT, bool BATCH>
static hipError_t launch2d_mfma(const StageArgs &a, hipStream_t s) {
    // every pointer the kernel dereferences must be set
    if (!a.opsfrag || a.ntiles <= 0 || a.ngroups < 8 || (a.ngroups & 7)) return hipErrorInvalidValue;
    if (BATCH ? (!a.batch || !a.tile_req) : (!a.qin || !a.qout || !a.res || !a.geo || !a.fgeo || !a.nbr))
        return hipErrorInvalidValue;
    hipLaunchKernelGGL((stage2d_mfma_kernel<N, MAT, BATCH>), dim3(a.ngroups), dim3(512), 0, s, a);
    return hipGetLastError();
}

template <int N, bool MAT, bool BATCH>
static int occupancy2d_mfma() {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, stage2d_mfma_kernel<N, MAT, BATCH>, 512, 0) != hipSuccess)
        return 1;
    return nb > 0 ? nb : 1;
}

#define DGW_ORDERS(X) X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8)

hipError_t launch_stage2d_mfma(int N, bool material, const StageArgs &a, hipStream_t s) {
#define DGW_CASE(n) \
    case n: return material ? launch2d_mfma<n, true, false>(a, s) : launch2d_mfma<n, false, false>(a, s);
    switch (N) {
        DGW_ORDERS(DGW_CASE)
        default: return hipErrorInvalidValue;
    }
#undef DGW_CASE
}

hipError_t launch_stage2d_batch(int N, bool material, const StageArgs &a, hipStream_t s) {
#define DGW_CASE(n) \
    case n: return material ? launch2d_mfma<n, true, true>(a, s) : launch2d_mfma<n, false, true>(a, s);
    switch (N) {
        DGW_ORDERS(DGW_CASE)
        default: return hipErrorInvalidValue;
    }
#undef DGW_CASE
}

int blocks_per_cu_2d_mfma(int N, bool material) {
#define DGW_CASE(n) \
    case n: return material ? occupancy2d_mfma<n, true, false>() : occupancy2d_mfma<n, false, false>();
    switch (N) {
        DGW_ORDERS(DGW_CASE)
        default: return 1;
    }
#undef DGW_CASE
}

int blocks_per_cu_2d_batch(int N, bool material) {
#define DGW_CASE(n) \
    case n: return material ? occupancy2d_mfma<n, true, true>() : occupancy2d_mfma<n, false, true>();
    switch (N) {
        DGW_ORDERS(DGW_CASE)
        default: return 1;
    }
#undef DGW_CASE
}

// Fragment-ordered copy of the fused operator [Dr | Ds | LIFT] for the A
// operand: out[(mt*KS + ks)*64 + l] = Op[16 mt + l%16][4 ks + l/16] (zero
// outside Np x Kd).  Returns the number of floats written (MT*KS*64).
int opsfrag2d(int N, const double *Dr, const double *Ds, const double *LIFT, float *out) {
    const int Np = (N + 1) * (N + 2) / 2, Nafp = 3 * (N + 1), Kd = 2 * Np + Nafp;
    const int KS = (Kd + 3) / 4, MT = (Np + 15) / 16;
    if (!out) return MT * KS * 64;
    for (int mt = 0; mt < MT; ++mt)
        for (int ks = 0; ks < KS; ++ks)
            for (int l = 0; l < 64; ++l) {
                // the 4x4x1 tail takes rows 16 mt + l%4 (see tail4_rows)
                const int row = 16 * mt + ((tail4_rows(N) && mt == MT - 1) ? l % 4 : l % 16), k = 4 * ks + l / 16;
                double v = 0.0;
                if (row < Np && k < Kd) {
                    if (k < Np)
                        v = Dr[row * Np + k];
                    else if (k < 2 * Np)
                        v = Ds[row * Np + (k - Np)];
                    else
                        v = LIFT[row * Nafp + (k - 2 * Np)];
                }
                out[(mt * KS + ks) * 64 + l] = (float)v;
            }
    return MT * KS * 64;
}

// The closed-form face node order used by the kernel, for the host's check
// against the reference element it built.
int face_node2d(int N, int f, int t) {
    auto lat = [N](int i, int j) { return j * (N + 1) - j * (j - 1) / 2 + i; };
    return f == 0 ? t : (f == 1 ? lat(N - t, t) : lat(0, N - t));
}

}  // namespace dgw
