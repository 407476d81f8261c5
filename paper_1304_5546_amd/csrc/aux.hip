// FP64 reductions (energy, error against the closed-form cavity mode), the
// on-device FP64 cavity-mode initialisation and the layout permutations
// between the caller's element-major and the internal node-major layout.
#include <hip/hip_runtime.h>

#include <cmath>

#include "device.hpp"

namespace dgw {

namespace {

constexpr int kRedThreads = 256;

// deterministic block reduction of one double per thread
__device__ double block_sum(double v, double *sh) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) sh[w] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int i = 0; i < kRedThreads / 64; ++i) s += sh[i];
    __syncthreads();
    return s;
}

// field value i as FP64, from the FP32 or the FP64 field array
template <bool D64, typename Args>
__device__ __forceinline__ double qval(const Args &a, size_t i) {
    if constexpr (D64)
        return a.q64[i];
    else
        return (double)a.q[i];
}

// one thread per element: sum_f w_f q_f^T M q_f J
template <bool D64>
__global__ void __launch_bounds__(kRedThreads) energy_kernel(ReduceArgs a) {
    __shared__ double sh[kRedThreads / 64];
    double acc = 0.0;
    for (int e = blockIdx.x * kRedThreads + threadIdx.x; e < a.K; e += gridDim.x * kRedThreads) {
        double ek = 0.0;
        for (int f = 0; f < a.nf; ++f) {
            double qf = 0.0;
            for (int i = 0; i < a.Np; ++i) {
                const double qi = qval<D64>(a, fidx(e, f, i, a.nf, a.Np, a.npp));
                double mq = 0.0;
                for (int j = 0; j < a.Np; ++j) mq += a.Mref[i * a.Np + j] * qval<D64>(a, fidx(e, f, j, a.nf, a.Np, a.npp));
                qf += qi * mq;
            }
            ek += (a.w ? a.w[tix(e, f, a.nf)] : 1.0) * qf;
        }
        acc += a.J[e] * ek;
    }
    const double s = block_sum(acc, sh);
    if (threadIdx.x == 0) a.partial[blockIdx.x] = s;
}

// Sum of the n per-block partials in index order (the order of the host sum
// of dgw_energy), scaled: one thread, so the result is bitwise that sum.
__global__ void sum_partials_kernel(const double *partial, int n, double scale, double *out) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += partial[i];
    *out = scale * s;
}

__device__ void cavity_exact(const CavityArgs &a, double x, double y, double z, double *out) {
    const double pi = M_PI;
    if (a.dim == 2) {
        const double w = pi * sqrt(double(a.m * a.m + a.n * a.n)) / sqrt(a.eps * a.mu);
        const double sx = sin(a.m * pi * x), cx = cos(a.m * pi * x);
        const double sy = sin(a.n * pi * y), cy = cos(a.n * pi * y);
        const double ct = cos(w * a.t), st = sin(w * a.t);
        out[0] = -(a.n * pi / (a.mu * w)) * sx * cy * st;
        out[1] = (a.m * pi / (a.mu * w)) * cx * sy * st;
        out[2] = sx * sy * ct;
    } else {
        // E = (Ax cx sy sz, Ay sx cy sz, Az sx sy cz) cos(wt), A = (n, -m, 0),
        // H = -(1/w) curl(E_spatial) sin(wt), w = pi sqrt(m^2+n^2+l^2)
        const double km = a.m * pi, kn = a.n * pi, kl = a.l * pi;
        const double w = sqrt(km * km + kn * kn + kl * kl);
        const double Ax = a.n, Ay = -a.m, Az = 0.0;
        const double sx = sin(km * x), cx = cos(km * x), sy = sin(kn * y), cy = cos(kn * y);
        const double sz = sin(kl * z), cz = cos(kl * z);
        const double ct = cos(w * a.t), st = sin(w * a.t);
        // curl of the spatial E
        const double cxE = (Az * kn - Ay * kl) * sx * cy * cz;
        const double cyE = (Ax * kl - Az * km) * cx * sy * cz;
        const double czE = (Ay * km - Ax * kn) * cx * cy * sz;
        out[0] = -cxE * st / w;
        out[1] = -cyE * st / w;
        out[2] = -czE * st / w;
        out[3] = Ax * cx * sy * sz * ct;
        out[4] = Ay * sx * cy * sz * ct;
        out[5] = Az * sx * sy * cz * ct;
    }
}

template <bool D64>
__global__ void cavity_init_kernel(CavityArgs a) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    const int nf = a.dim == 2 ? 3 : 6;
    if (e >= a.Kp) return;
    for (int i = 0; i < a.Np; ++i) {
        double out[6] = {0, 0, 0, 0, 0, 0};
        if (e < a.K) {
            const size_t p = tix(e, i, a.Np);
            cavity_exact(a, a.x[p], a.y[p], a.dim == 3 ? a.z[p] : 0.0, out);
        }
        for (int f = 0; f < nf; ++f) {
            const size_t p = fidx(e, f, i, nf, a.Np, a.npp);
            if constexpr (D64)
                a.q64[p] = out[f];
            else
                a.q[p] = (float)out[f];
        }
    }
}

// one thread per element; accumulates ||q - q_exact||^2_M and ||q_exact||^2_M
// (the closed form is re-evaluated inside the M product instead of being
// stored, keeping the kernel free of large per-lane arrays)
template <bool D64>
__global__ void __launch_bounds__(kRedThreads) cavity_error_kernel(CavityArgs a) {
    __shared__ double sh[kRedThreads / 64];
    const int nf = a.dim == 2 ? 3 : 6;
    double num = 0.0, den = 0.0;
    for (int e = blockIdx.x * kRedThreads + threadIdx.x; e < a.K; e += gridDim.x * kRedThreads) {
        double nk = 0.0, dk = 0.0;
        for (int i = 0; i < a.Np; ++i) {
            const size_t pi = tix(e, i, a.Np);
            double exi[6], di[6], md[6] = {0, 0, 0, 0, 0, 0}, mx[6] = {0, 0, 0, 0, 0, 0};
            cavity_exact(a, a.x[pi], a.y[pi], a.dim == 3 ? a.z[pi] : 0.0, exi);
            for (int f = 0; f < nf; ++f) di[f] = qval<D64>(a, fidx(e, f, i, nf, a.Np, a.npp)) - exi[f];
            for (int j = 0; j < a.Np; ++j) {
                const size_t pj = tix(e, j, a.Np);
                double exj[6];
                cavity_exact(a, a.x[pj], a.y[pj], a.dim == 3 ? a.z[pj] : 0.0, exj);
                const double Mij = a.Mref[i * a.Np + j];
                for (int f = 0; f < nf; ++f) {
                    md[f] += Mij * (qval<D64>(a, fidx(e, f, j, nf, a.Np, a.npp)) - exj[f]);
                    mx[f] += Mij * exj[f];
                }
            }
            for (int f = 0; f < nf; ++f) {
                nk += di[f] * md[f];
                dk += exi[f] * mx[f];
            }
        }
        num += a.J[e] * nk;
        den += a.J[e] * dk;
    }
    const double s1 = block_sum(num, sh);
    const double s2 = block_sum(den, sh);
    if (threadIdx.x == 0) {
        a.partial[2 * blockIdx.x] = s1;
        a.partial[2 * blockIdx.x + 1] = s2;
    }
}

// element-major <-> tiled copy of one field array (every destination slot
// written; pad nodes 0)
__global__ void relayout_kernel(const float *src, float *dst, int Kp, int Np, int nf, int npp_src, int npp_dst) {
    const int nd = npp_dst ? npp_dst : Np;
    const size_t total = (size_t)Kp * nf * nd;
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (size_t)gridDim.x * blockDim.x) {
        const int n = int(t % nd);
        const int f = int((t / nd) % nf);
        const int64_t e = int64_t(t / ((size_t)nd * nf));
        dst[fidx(e, f, n, nf, Np, npp_dst)] = n < Np ? src[fidx(e, f, n, nf, Np, npp_src)] : 0.0f;
    }
}

// every slot of the internal array is written (padding elements and pad
// nodes with 0)
__global__ void to_internal_kernel(const float *src, float *dst, const int *perm, int K, int Kp, int Np, int nf,
                                   int npp) {
    const size_t total = npp ? (size_t)Kp * nf * npp : (size_t)nf * Np * Kp;
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (size_t)gridDim.x * blockDim.x) {
        int e, n, f;
        if (npp) {
            n = int(t % npp);
            f = int((t / npp) % nf);
            e = int(t / ((size_t)npp * nf));
        } else {
            const int rows = nf * Np;
            e = int((t / ((size_t)64 * rows)) * 64 + (t & 63));
            const int row = int((t / 64) % rows);
            n = row % Np;
            f = row / Np;
        }
        dst[t] = (e < K && n < Np) ? src[((size_t)f * K + perm[e]) * Np + n] : 0.0f;
    }
}

__global__ void to_caller_kernel(const float *src, float *dst, const int *perm, int K, int Kp, int Np, int nf,
                                 int npp) {
    const size_t total = (size_t)nf * Np * K;
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (size_t)gridDim.x * blockDim.x) {
        const int e = int(t % K);
        const size_t fn = t / K;
        const int n = int(fn % Np), f = int(fn / Np);
        dst[((size_t)f * K + perm[e]) * Np + n] = src[fidx(e, f, n, nf, Np, npp)];
    }
}

}  // namespace

// Each launch reads (or writes) q64 when it is set, else q.
hipError_t launch_energy(const ReduceArgs &a, int nblocks, hipStream_t s) {
    if (!a.q && !a.q64) return hipErrorInvalidValue;
    if (a.q64)
        hipLaunchKernelGGL(energy_kernel<true>, dim3(nblocks), dim3(kRedThreads), 0, s, a);
    else
        hipLaunchKernelGGL(energy_kernel<false>, dim3(nblocks), dim3(kRedThreads), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_sum_partials(const double *partial, int n, double scale, double *out, hipStream_t s) {
    if (!partial || !out || n < 0) return hipErrorInvalidValue;
    hipLaunchKernelGGL(sum_partials_kernel, dim3(1), dim3(64), 0, s, partial, n, scale, out);
    return hipGetLastError();
}

hipError_t launch_cavity_init(const CavityArgs &a, hipStream_t s) {
    if (!a.q && !a.q64) return hipErrorInvalidValue;
    if (a.q64)
        hipLaunchKernelGGL(cavity_init_kernel<true>, dim3((a.Kp + 255) / 256), dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL(cavity_init_kernel<false>, dim3((a.Kp + 255) / 256), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_cavity_error(const CavityArgs &a, int nblocks, hipStream_t s) {
    if (!a.q && !a.q64) return hipErrorInvalidValue;
    if (a.q64)
        hipLaunchKernelGGL(cavity_error_kernel<true>, dim3(nblocks), dim3(kRedThreads), 0, s, a);
    else
        hipLaunchKernelGGL(cavity_error_kernel<false>, dim3(nblocks), dim3(kRedThreads), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_relayout(const float *src, float *dst, int Kp, int Np, int nf, int npp_src, int npp_dst,
                           hipStream_t s) {
    if (!src || !dst || src == dst) return hipErrorInvalidValue;
    hipLaunchKernelGGL(relayout_kernel, dim3(2048), dim3(256), 0, s, src, dst, Kp, Np, nf, npp_src, npp_dst);
    return hipGetLastError();
}

hipError_t launch_to_internal(const float *src, float *dst, const int *perm, int K, int Kp, int Np, int nf, int npp,
                              hipStream_t s) {
    hipLaunchKernelGGL(to_internal_kernel, dim3(2048), dim3(256), 0, s, src, dst, perm, K, Kp, Np, nf, npp);
    return hipGetLastError();
}

hipError_t launch_to_caller(const float *src, float *dst, const int *perm, int K, int Kp, int Np, int nf, int npp,
                            hipStream_t s) {
    hipLaunchKernelGGL(to_caller_kernel, dim3(2048), dim3(256), 0, s, src, dst, perm, K, Kp, Np, nf, npp);
    return hipGetLastError();
}

}  // namespace dgw
