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

// Several two-qubit gates on disjoint or overlapping pairs inside one tile of 2^T
// amplitudes, T = W + H <= 12: the tile's index bits are [0, W) and [hb, hb + H)
// (local index l -> l mod 2^W + (l >> W) 2^hb), the other n - T bits number the
// tiles.  The tile is loaded into LDS once, the gates are applied in order (local bit
// positions a[g], b[g]; matrix on the local index b_a + 2 b_b), and it is written back:
// one pass over the state for a whole group of gates.
constexpr int TILE_GATES_MAX = 6;

template <typename R>
struct TileGates {
    Mat4<R> m[TILE_GATES_MAX];
    int a[TILE_GATES_MAX], b[TILE_GATES_MAX];
    int ng;
};

template <typename R, int T>
__global__ void __launch_bounds__(256)
k_gates_tile(cx<R>* __restrict__ psi, int W, int hb, int H, TileGates<R> G) {
    constexpr uint32_t size = 1u << T;
    constexpr int PER = size >= 256 ? (int)(size / 256) : 1;
    __shared__ cx<R> t[size];
    const uint32_t tid = threadIdx.x;
    const uint64_t tile = blockIdx.x;
    const uint64_t tmid = tile & ((1ull << (hb - W)) - 1ull);
    const uint64_t ttop = tile >> (hb - W);
    cx<R>* base = psi + (tmid << W) + (ttop << (hb + H));
    const uint32_t wm = (1u << W) - 1u;
    // all of a thread's loads are issued before any is written to LDS
    {
        cx<R> v[PER];
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            const uint32_t i = tid + 256u * j;
            if (i < size) v[j] = base[(i & wm) + ((size_t)(i >> W) << hb)];
        }
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            const uint32_t i = tid + 256u * j;
            if (i < size) t[i] = v[j];
        }
    }
    __syncthreads();
    for (int g = 0; g < G.ng; ++g) {
        const int a = G.a[g], b = G.b[g];
        const int lo = a < b ? a : b, hi = a < b ? b : a;
        const uint32_t llo = (1u << lo) - 1u, lhi = (1u << hi) - 1u;
        for (uint32_t k = tid; k < (size >> 2); k += 256) {
            uint32_t q = (k & llo) | ((k & ~llo) << 1);
            q = (q & lhi) | ((q & ~lhi) << 1);
            const uint32_t idx[4] = {q, q | (1u << a), q | (1u << b), q | (1u << a) | (1u << b)};
            cx<R> in[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) in[j] = t[idx[j]];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                R sr = R(0), si = R(0);
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    const cx<R> m = G.m[g].u[4 * r + c];
                    sr += m.re * in[c].re - m.im * in[c].im;
                    si += m.re * in[c].im + m.im * in[c].re;
                }
                cx<R> o;
                o.re = sr;
                o.im = si;
                t[idx[r]] = o;
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int j = 0; j < PER; ++j) {
        const uint32_t i = tid + 256u * j;
        if (i < size) base[(i & wm) + ((size_t)(i >> W) << hb)] = t[i];
    }
}

template <typename R>
hipError_t gates_tile_t(void* psi, int n, int W, int hb, int H, int ng, const int* a, const int* b,
                        const double* m32, hipStream_t st) {
    TileGates<R> G{};
    G.ng = ng;
    for (int g = 0; g < ng; ++g) {
        G.a[g] = a[g];
        G.b[g] = b[g];
        for (int k = 0; k < 16; ++k) {
            G.m[g].u[k].re = (R)m32[32 * g + 2 * k];
            G.m[g].u[k].im = (R)m32[32 * g + 2 * k + 1];
        }
    }
    const uint64_t tiles = 1ull << (n - W - H);
    switch (W + H) {
#define PW_TG(T) \
    case T: hipLaunchKernelGGL((k_gates_tile<R, T>), dim3((unsigned)tiles), dim3(256), 0, st, (cx<R>*)psi, W, hb, H, G); break;
        PW_TG(2) PW_TG(3) PW_TG(4) PW_TG(5) PW_TG(6) PW_TG(7) PW_TG(8) PW_TG(9) PW_TG(10) PW_TG(11) PW_TG(12)
#undef PW_TG
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
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

hipError_t apply_gates_tile(bool dbl, void* psi, int n, int W, int hb, int H, int ng, const int* a, const int* b,
                            const double* m32, hipStream_t st) {
    if (ng < 1 || ng > TILE_GATES_MAX || W < 0 || H < 0 || W + H > 12 || W + H > n || (H > 0 && (hb < W || hb + H > n)))
        return hipErrorInvalidValue;
    if (H == 0) hb = W;
    for (int g = 0; g < ng; ++g)
        if (a[g] < 0 || b[g] < 0 || a[g] >= W + H || b[g] >= W + H || a[g] == b[g]) return hipErrorInvalidValue;
    return dbl ? gates_tile_t<double>(psi, n, W, hb, H, ng, a, b, m32, st)
               : gates_tile_t<float>(psi, n, W, hb, H, ng, a, b, m32, st);
}

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

namespace {
// dst = src converted amplitude by amplitude (complex128 <-> complex64, round to nearest).
template <typename S, typename D>
__global__ void __launch_bounds__(256) k_convert(const cx<S>* __restrict__ src, cx<D>* __restrict__ dst, uint64_t d) {
    const uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= d) return;
    const cx<S> v = src[i];
    cx<D> o;
    o.re = (D)v.re;
    o.im = (D)v.im;
    dst[i] = o;
}
}  // namespace

hipError_t convert_state(bool src_dbl, const void* src, void* dst, int n, hipStream_t st) {
    const uint64_t d = 1ull << n;
    const dim3 grid((unsigned)((d + 255) / 256));
    if (src_dbl)
        hipLaunchKernelGGL((k_convert<double, float>), grid, dim3(256), 0, st, (const cx<double>*)src, (cx<float>*)dst, d);
    else
        hipLaunchKernelGGL((k_convert<float, double>), grid, dim3(256), 0, st, (const cx<float>*)src, (cx<double>*)dst, d);
    return hipGetLastError();
}

hipError_t apply_gate2(bool dbl, void* psi, int n, int q0, int q1, const double* m16, hipStream_t st) {
    return dbl ? gate2_t<double>(psi, n, q0, q1, m16, st) : gate2_t<float>(psi, n, q0, q1, m16, st);
}

hipError_t apply_diag(bool dbl, void* psi, int n, int q, const double* d2, hipStream_t st) {
    return dbl ? diag_t<double>(psi, n, q, d2, st) : diag_t<float>(psi, n, q, d2, st);
}

}  // namespace pw
