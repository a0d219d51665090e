// Draws of X-bitstrings for the Monte Carlo estimators.
//
//  * Uniform over F_2^N \ {0} (the paper's Monte Carlo section).
//  * Exact x-marginal p(x) = sum_z c_{x,z}^2 / d = sum_b q(b) q(b^x), q = |psi|^2:
//    x = b1 ^ b2 with b1, b2 independent draws from q, redrawn while x = 0.
//    Draws from q invert an FP64 inclusive prefix sum of q.  A draw still 0 after
//    64 attempts takes the pair directly from its law given b1 != b2 (b1 from
//    q (T - q), a second prefix sum, then b2 from q without b1), so the output
//    follows p(x) / (1 - p(0)) exactly whatever p(0) < 1.
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

// The weight summed into a prefix table: q(b) = |psi(b)|^2, or with W the weight
// q(b) (T - q(b)) of b as the first element of a pair of distinct draws, T the total
// of q (the last entry of the finished q table).
template <typename R, bool W>
__device__ __forceinline__ double cdf_weight(const cx<R>* __restrict__ psi, uint64_t b, const double* __restrict__ qtot) {
    const cx<R> v = psi[b];
    const double re = (double)v.re, im = (double)v.im;
    const double q = re * re + im * im;
    if constexpr (W) return q * (*qtot - q);
    return q;
}

// Phase 1: fixed-order sum of the weights over each chunk.
template <typename R, bool W>
__global__ void __launch_bounds__(256) k_cdf_sums(const cx<R>* __restrict__ psi, uint64_t d, double* __restrict__ blk,
                                                  const double* __restrict__ qtot) {
    __shared__ double sh[256];
    const uint64_t base = (uint64_t)blockIdx.x * CDF_CHUNK;
    double s = 0.0;
    // thread t owns the 16 consecutive amplitudes [base + 16t, base + 16t + 16)
    for (int j = 0; j < CDF_CHUNK / 256; ++j) {
        const uint64_t b = base + (uint64_t)threadIdx.x * (CDF_CHUNK / 256) + j;
        if (b < d) s += cdf_weight<R, W>(psi, b, qtot);
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
template <typename R, bool W>
__global__ void __launch_bounds__(256)
k_cdf_final(const cx<R>* __restrict__ psi, uint64_t d, const double* __restrict__ blk, double* __restrict__ cdf,
            const double* __restrict__ qtot) {
    __shared__ double sh[256];
    constexpr int PER = CDF_CHUNK / 256;
    const uint64_t base = (uint64_t)blockIdx.x * CDF_CHUNK + (uint64_t)threadIdx.x * PER;
    double q[PER];
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < PER; ++j) {
        const uint64_t b = base + j;
        s += b < d ? cdf_weight<R, W>(psi, b, qtot) : 0.0;
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

// Smallest k in [lo, hi] with C[k] > t, or hi when there is none.
__device__ __forceinline__ uint64_t upper_bound(const double* __restrict__ C, uint64_t lo, uint64_t hi, double t) {
    while (lo < hi) {
        const uint64_t mid = lo + ((hi - lo) >> 1);
        if (C[mid] > t) hi = mid;
        else lo = mid + 1;
    }
    return lo;
}

// b1 from the table of q (T - q), then b2 from q with b1's own interval of C taken
// out: the point u2 (T - q(b1)) of the remaining mass, searched below b1 or, shifted
// past b1's interval, above it.  b2 != b1 by construction; 0 only when the q (T - q)
// table is empty (q a point mass).
__device__ __forceinline__ uint64_t distinct_pair(const double* __restrict__ C, const double* __restrict__ Cw,
                                                  uint64_t d, double u1, double u2) {
    const double T = C[d - 1], Tw = Cw[d - 1];
    if (!(Tw > 0.0)) return 0;
    const uint64_t b1 = upper_bound(Cw, 0, d - 1, u1 * Tw);
    const double below = b1 ? C[b1 - 1] : 0.0;
    const double t = u2 * (T - (C[b1] - below));
    const uint64_t b2 = (b1 > 0 && (t < below || b1 == d - 1)) ? upper_bound(C, 0, b1 - 1, t)
                                                                : upper_bound(C, b1 + 1, d - 1, C[b1] + (t - below));
    return b1 ^ b2;
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
        x = upper_bound(cdf, 0, d - 1, u1 * T) ^ upper_bound(cdf, 0, d - 1, u2 * T);
    }
    if (x == 0) {
        uint64_t W0, W1;
        words(seed, offset + (uint64_t)i, (uint32_t)MAX_ATTEMPTS, STREAM_MARGINAL, W0, W1);
        x = distinct_pair(cdf, cdf + d, d, (double)(W0 >> 11) * 0x1.0p-53, (double)(W1 >> 11) * 0x1.0p-53);
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

template <typename R, bool W>
hipError_t build_table(const cx<R>* psi, uint64_t d, unsigned nb, double* tab, double* blk, const double* qtot,
                       hipStream_t st) {
    hipLaunchKernelGGL((k_cdf_sums<R, W>), dim3(nb), dim3(256), 0, st, psi, d, blk, qtot);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_cdf_scan_blocks, dim3(1), dim3(256), 0, st, blk, (int64_t)nb);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_cdf_final<R, W>), dim3(nb), dim3(256), 0, st, psi, d, blk, tab, qtot);
    return hipGetLastError();
}

template <typename R>
hipError_t build_tables(const cx<R>* psi, int n, double* d_cdf, double* d_blk, hipStream_t st) {
    const uint64_t d = 1ull << n;
    const unsigned nb = (unsigned)cdf_blk_elems(n);
    hipError_t e = build_table<R, false>(psi, d, nb, d_cdf, d_blk, nullptr, st);
    if (e != hipSuccess) return e;
    return build_table<R, true>(psi, d, nb, d_cdf + d, d_blk + nb, d_cdf + (d - 1), st);
}

// d_cdf holds 2 * 2^n doubles (the prefix sums of q = |psi|^2, then those of
// q (T - q)), d_blk 2 * cdf_blk_elems(n) doubles of chunk offsets.
hipError_t build_cdf(bool dbl, const void* psi, int n, double* d_cdf, double* d_blk, hipStream_t st) {
    return dbl ? build_tables((const cx<double>*)psi, n, d_cdf, d_blk, st)
               : build_tables((const cx<float>*)psi, n, d_cdf, d_blk, st);
}

hipError_t sample_marginal(int n, const double* d_cdf, uint64_t seed, uint64_t offset, int64_t count, uint64_t* d_xs,
                           hipStream_t st, const uint64_t* d_off) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_marginal, dim3((unsigned)((count + 63) / 64)), dim3(64), 0, st, n, d_cdf, seed, offset, d_off,
                       count, d_xs);
    return hipGetLastError();
}

}  // namespace pw
