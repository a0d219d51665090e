// Draws of X-bitstrings for the Monte Carlo estimators.
//
//  * Uniform over F_2^N \ {0} (the paper's Monte Carlo section).
//  * Exact x-marginal p(x) = sum_z c_{x,z}^2 / d = sum_b q(b) q(b^x), q = |psi|^2:
//    x = b1 ^ b2 with b1, b2 independent draws from q, redrawn while x = 0.
//    Draws from q invert an FP64 inclusive prefix sum of q.
//
// Random words come from Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) with
// counter (i_lo, i_hi, attempt, stream) and key (seed_lo, seed_hi), so the
// list of sample i is reproducible and independent of batching.
#include "common.h"
#include "philox.h"

namespace pw {
namespace {

constexpr int MAX_ATTEMPTS = 64;
constexpr int CDF_CHUNK = 4096;                      // amplitudes per scan workgroup

__device__ __forceinline__ void words(uint64_t seed, uint64_t g, uint32_t attempt, uint32_t stream, uint64_t& W0,
                                      uint64_t& W1) {
    philox_words(seed, g, attempt, stream, W0, W1);
}

__global__ void k_uniform(int n, uint64_t seed, uint64_t offset, const uint64_t* __restrict__ d_off, int64_t count,
                          uint64_t* __restrict__ xs) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= count) return;
    if (d_off) offset += *d_off;
    uint64_t W0, W1;
    words(seed, offset + (uint64_t)i, 0u, STREAM_UNIFORM, W0, W1);
    xs[i] = 1ull + __umul64hi(W0, (1ull << n) - 1ull);
}

// Phase 1: fixed-order sum of q over each chunk.
template <typename R>
__global__ void __launch_bounds__(256) k_cdf_sums(const cx<R>* __restrict__ psi, uint64_t d, double* __restrict__ blk) {
    __shared__ double sh[256];
    const uint64_t base = (uint64_t)blockIdx.x * CDF_CHUNK;
    double s = 0.0;
    // thread t owns the 16 consecutive amplitudes [base + 16t, base + 16t + 16)
    for (int j = 0; j < CDF_CHUNK / 256; ++j) {
        const uint64_t b = base + (uint64_t)threadIdx.x * (CDF_CHUNK / 256) + j;
        if (b < d) {
            const cx<R> v = psi[b];
            const double re = (double)v.re, im = (double)v.im;
            s += re * re + im * im;
        }
    }
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) sh[threadIdx.x] += sh[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) blk[blockIdx.x] = sh[0];
}

// Inclusive scan of v[0..n) held one per thread in sh[0..256) (Hillis-Steele).
__device__ __forceinline__ double block_incl_scan(double v, double* sh) {
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
        const double t = (int)threadIdx.x >= off ? sh[threadIdx.x - off] : 0.0;
        __syncthreads();
        sh[threadIdx.x] += t;
        __syncthreads();
    }
    return sh[threadIdx.x];
}

// Phase 2: exclusive scan of the chunk sums, one workgroup, 256 at a time.
__global__ void __launch_bounds__(256) k_cdf_scan_blocks(double* __restrict__ blk, int64_t nblk) {
    __shared__ double sh[256];
    double carry = 0.0;
    for (int64_t base = 0; base < nblk; base += 256) {
        const int64_t i = base + threadIdx.x;
        const double v = i < nblk ? blk[i] : 0.0;
        const double inc = block_incl_scan(v, sh);
        if (i < nblk) blk[i] = carry + inc - v;
        const double tot = sh[255];
        __syncthreads();
        carry += tot;
    }
}

// Phase 3: inclusive scan inside each chunk plus the chunk's offset.
template <typename R>
__global__ void __launch_bounds__(256)
k_cdf_final(const cx<R>* __restrict__ psi, uint64_t d, const double* __restrict__ blk, double* __restrict__ cdf) {
    __shared__ double sh[256];
    constexpr int PER = CDF_CHUNK / 256;
    const uint64_t base = (uint64_t)blockIdx.x * CDF_CHUNK + (uint64_t)threadIdx.x * PER;
    double q[PER];
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < PER; ++j) {
        const uint64_t b = base + j;
        double v = 0.0;
        if (b < d) {
            const cx<R> a = psi[b];
            const double re = (double)a.re, im = (double)a.im;
            v = re * re + im * im;
        }
        s += v;
        q[j] = s;
    }
    const double inc = block_incl_scan(s, sh);
    const double off = blk[blockIdx.x] + (inc - s);
#pragma unroll
    for (int j = 0; j < PER; ++j) {
        const uint64_t b = base + j;
        if (b < d) cdf[b] = off + q[j];
    }
}

__device__ __forceinline__ uint64_t upper_bound(const double* __restrict__ C, uint64_t d, double t) {
    uint64_t lo = 0, hi = d - 1;
    while (lo < hi) {
        const uint64_t mid = lo + ((hi - lo) >> 1);
        if (C[mid] > t) hi = mid;
        else lo = mid + 1;
    }
    return lo;
}

__global__ void k_marginal(int n, const double* __restrict__ cdf, uint64_t seed, uint64_t offset,
                           const uint64_t* __restrict__ d_off, int64_t count, uint64_t* __restrict__ xs) {
    const int64_t i = (int64_t)blockIdx.x * 64 + threadIdx.x;
    if (i >= count) return;
    if (d_off) offset += *d_off;
    const uint64_t d = 1ull << n;
    const double T = cdf[d - 1];
    uint64_t x = 0;
    for (int a = 0; a < MAX_ATTEMPTS && x == 0; ++a) {
        uint64_t W0, W1;
        words(seed, offset + (uint64_t)i, (uint32_t)a, STREAM_MARGINAL, W0, W1);
        const double u1 = (double)(W0 >> 11) * 0x1.0p-53, u2 = (double)(W1 >> 11) * 0x1.0p-53;
        x = upper_bound(cdf, d, u1 * T) ^ upper_bound(cdf, d, u2 * T);
    }
    xs[i] = x;
}

__global__ void k_bump(uint64_t* __restrict__ ctr, uint64_t v) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *ctr += v;
}

}  // namespace

hipError_t bump_counter(uint64_t* d_ctr, uint64_t v, hipStream_t st) {
    hipLaunchKernelGGL(k_bump, dim3(1), dim3(64), 0, st, d_ctr, v);
    return hipGetLastError();
}

hipError_t sample_uniform(int n, uint64_t seed, uint64_t offset, int64_t count, uint64_t* d_xs, hipStream_t st,
                          const uint64_t* d_off) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_uniform, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, n, seed, offset, d_off, count,
                       d_xs);
    return hipGetLastError();
}

size_t cdf_blk_elems(int n) {
    const uint64_t d = 1ull << n;
    return (size_t)((d + CDF_CHUNK - 1) / CDF_CHUNK);
}

hipError_t build_cdf(bool dbl, const void* psi, int n, double* d_cdf, double* d_blk, hipStream_t st) {
    const uint64_t d = 1ull << n;
    const unsigned nb = (unsigned)cdf_blk_elems(n);
    if (dbl)
        hipLaunchKernelGGL(k_cdf_sums<double>, dim3(nb), dim3(256), 0, st, (const cx<double>*)psi, d, d_blk);
    else
        hipLaunchKernelGGL(k_cdf_sums<float>, dim3(nb), dim3(256), 0, st, (const cx<float>*)psi, d, d_blk);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_cdf_scan_blocks, dim3(1), dim3(256), 0, st, d_blk, (int64_t)nb);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (dbl)
        hipLaunchKernelGGL(k_cdf_final<double>, dim3(nb), dim3(256), 0, st, (const cx<double>*)psi, d, d_blk, d_cdf);
    else
        hipLaunchKernelGGL(k_cdf_final<float>, dim3(nb), dim3(256), 0, st, (const cx<float>*)psi, d, d_blk, d_cdf);
    return hipGetLastError();
}

hipError_t sample_marginal(int n, const double* d_cdf, uint64_t seed, uint64_t offset, int64_t count, uint64_t* d_xs,
                           hipStream_t st, const uint64_t* d_off) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_marginal, dim3((unsigned)((count + 63) / 64)), dim3(64), 0, st, n, d_cdf, seed, offset, d_off,
                       count, d_xs);
    return hipGetLastError();
}

}  // namespace pw
