// State kernels: FP64 norm check on bind, and gate application for Clifford
// preconditioning and circuit-state preparation (Clifford preconditioning
// section: a brick-wall circuit of random two-qubit Cliffords applied to the
// state before sampling; T = diag(1, e^{i pi/4}) for T-doped circuits).
#include "common.h"

namespace pw {
namespace {

constexpr int NORM_CHUNK = 1 << 14;   // amplitudes per norm workgroup

template <typename R>
__global__ void __launch_bounds__(256)
k_norm_parts(const cx<R>* __restrict__ psi, uint64_t d, double* __restrict__ part, unsigned* __restrict__ bad) {
    __shared__ double sh[256];
    const uint64_t base = (uint64_t)blockIdx.x * NORM_CHUNK;
    double s = 0.0;
    unsigned nonfinite = 0u;
    for (uint64_t i = base + threadIdx.x; i < base + NORM_CHUNK && i < d; i += 256) {
        const cx<R> v = psi[i];
        const double re = (double)v.re, im = (double)v.im;
        if (!isfinite(re) || !isfinite(im)) nonfinite = 1u;
        s += re * re + im * im;
    }
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) sh[threadIdx.x] += sh[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
    if (nonfinite) atomicOr(bad, 1u);
}

__global__ void __launch_bounds__(256) k_norm_final(const double* __restrict__ part, int np, double* __restrict__ out) {
    __shared__ double sh[256];
    double s = 0.0;
    for (int i = threadIdx.x; i < np; i += 256) s += part[i];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) sh[threadIdx.x] += sh[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = sh[0];
}

template <typename R>
struct Mat4 {
    cx<R> u[16];
};

// One thread per amplitude quadruple {b, b|m0, b|m1, b|m0|m1} with b_{q0} = b_{q1} = 0.
template <typename R>
__global__ void __launch_bounds__(256)
k_gate2(cx<R>* __restrict__ psi, uint64_t nquad, int qlo, int qhi, int q0, int q1, Mat4<R> U) {
    const uint64_t t = (uint64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= nquad) return;
    const uint64_t llo = (1ull << qlo) - 1ull;
    uint64_t b = (t & llo) | ((t & ~llo) << 1);
    const uint64_t lhi = (1ull << qhi) - 1ull;
    b = (b & lhi) | ((b & ~lhi) << 1);
    const uint64_t m0 = 1ull << q0, m1 = 1ull << q1;
    const uint64_t idx[4] = {b, b | m0, b | m1, b | m0 | m1};
    cx<R> in[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) in[j] = psi[idx[j]];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        R sr = R(0), si = R(0);
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const cx<R> m = U.u[4 * r + c];
            sr += m.re * in[c].re - m.im * in[c].im;
            si += m.re * in[c].im + m.im * in[c].re;
        }
        cx<R> o;
        o.re = sr;
        o.im = si;
        psi[idx[r]] = o;
    }
}

template <typename R>
__global__ void __launch_bounds__(256)
k_diag(cx<R>* __restrict__ psi, uint64_t d, int q, cx<R> d0, cx<R> d1) {
    const uint64_t b = (uint64_t)blockIdx.x * 256 + threadIdx.x;
    if (b >= d) return;
    const cx<R> f = ((b >> q) & 1ull) ? d1 : d0;
    const cx<R> v = psi[b];
    cx<R> o;
    o.re = f.re * v.re - f.im * v.im;
    o.im = f.re * v.im + f.im * v.re;
    psi[b] = o;
}

template <typename R>
hipError_t gate2_t(void* psi, int n, int q0, int q1, const double* m16, hipStream_t st) {
    Mat4<R> U;
    for (int i = 0; i < 16; ++i) {
        U.u[i].re = (R)m16[2 * i];
        U.u[i].im = (R)m16[2 * i + 1];
    }
    const uint64_t nquad = 1ull << (n - 2);
    const int qlo = q0 < q1 ? q0 : q1, qhi = q0 < q1 ? q1 : q0;
    hipLaunchKernelGGL(k_gate2<R>, dim3((unsigned)((nquad + 255) / 256)), dim3(256), 0, st, (cx<R>*)psi, nquad, qlo,
                       qhi, q0, q1, U);
    return hipGetLastError();
}

template <typename R>
hipError_t diag_t(void* psi, int n, int q, const double* d2, hipStream_t st) {
    cx<R> a, b;
    a.re = (R)d2[0];
    a.im = (R)d2[1];
    b.re = (R)d2[2];
    b.im = (R)d2[3];
    const uint64_t d = 1ull << n;
    hipLaunchKernelGGL(k_diag<R>, dim3((unsigned)((d + 255) / 256)), dim3(256), 0, st, (cx<R>*)psi, d, q, a, b);
    return hipGetLastError();
}

}  // namespace

int norm2_parts(int n) {
    const uint64_t d = 1ull << n;
    return (int)((d + NORM_CHUNK - 1) / NORM_CHUNK);
}

hipError_t norm2(bool dbl, const void* psi, int n, double* d_partial, int nparts, double* d_out, unsigned* d_bad,
                 hipStream_t st) {
    const uint64_t d = 1ull << n;
    if (dbl)
        hipLaunchKernelGGL(k_norm_parts<double>, dim3(nparts), dim3(256), 0, st, (const cx<double>*)psi, d, d_partial,
                           d_bad);
    else
        hipLaunchKernelGGL(k_norm_parts<float>, dim3(nparts), dim3(256), 0, st, (const cx<float>*)psi, d, d_partial,
                           d_bad);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_norm_final, dim3(1), dim3(256), 0, st, d_partial, nparts, d_out);
    return hipGetLastError();
}

hipError_t apply_gate2(bool dbl, void* psi, int n, int q0, int q1, const double* m16, hipStream_t st) {
    return dbl ? gate2_t<double>(psi, n, q0, q1, m16, st) : gate2_t<float>(psi, n, q0, q1, m16, st);
}

hipError_t apply_diag(bool dbl, void* psi, int n, int q, const double* d2, hipStream_t st) {
    return dbl ? diag_t<double>(psi, n, q, d2, st) : diag_t<float>(psi, n, q, d2, st);
}

}  // namespace pw
