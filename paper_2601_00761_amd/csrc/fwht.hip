// Fused product + fast Walsh-Hadamard transform + reductions for families of
// Pauli strings (FWHT section and Algorithm 1 of Xiao & Ryu).
//
// For x != 0 the product f_x(b) = conj(psi(b)) psi(b^x) obeys f_x(b^x) = conj f_x(b),
// so with p the top set bit of x the half-size transform
//     G(z') = sum_{b : b_p = 0} (-1)^{z.b} f_x(b)          (2^(n-1) points)
// carries the whole family: |F_x(z)| is 2|Re G(z')| when x.z is even and
// 2|Im G(z')| when it is odd (z' = z without bit p).  For x = 0 the real vector
// q = |psi|^2 is packed as q(b') + i q(b' + 2^(n-1)) and F_0 = Re G +- Im G.
// Every family therefore costs one complex transform of 2^(n-1) points.
//
// Transform schedule on gfx950.  A tile of 2^K points lives in one workgroup:
// each of the 2^TL threads keeps 2^RL points in registers, radix-2 stages over
// the register bits run in registers, and an LDS exchange (padded one element in
// sixteen against bank conflicts) re-maps another block of RL index bits into
// registers.  Small states (n - 1 <= 13 single / 12 double) run the whole
// transform and the reductions in one workgroup per family.  Larger states use a
// first pass over the low 12 index bits (contiguous tiles, products formed at
// load time, coalesced) and column passes over the remaining bits (tiles of
// 2^s rows by 2^w >= 128-byte columns, coalesced); the last column pass reduces
// in registers and never writes the spectrum back.  Per-workgroup FP64 partials
// are summed per family in a fixed order by a separate finalize kernel, so
// results are bitwise reproducible.
#include "common.h"
#include <math.h>

namespace pw {
namespace {

template <typename R> struct Math;
template <> struct Math<float> {
    static __device__ __forceinline__ float lg2(float v) { return __log2f(v); }
};
template <> struct Math<double> {
    static __device__ __forceinline__ double lg2(double v) { return log2(v); }
};

__device__ __forceinline__ uint32_t win_idx(uint32_t tid, uint32_t j, int a, int rl) {
    return (tid & ((1u << a) - 1u)) | (j << a) | ((tid >> a) << (a + rl));
}
__device__ __forceinline__ uint32_t padi(uint32_t i) { return i + (i >> 4); }

template <int K> struct Lds { static constexpr int elems = (1 << K) + ((1 << K) >> 4); };

// Radix-2 butterflies (u, v) -> (u + v, u - v) over register bits [b0, b1).
template <typename R, int RL>
__device__ __forceinline__ void reg_stages(R (&re)[1 << RL], R (&im)[1 << RL], int b0, int b1) {
#pragma unroll
    for (int b = 0; b < RL; ++b) {
        if (b >= b0 && b < b1) {
#pragma unroll
            for (int j = 0; j < (1 << RL); ++j) {
                if (!(j & (1 << b))) {
                    const int k = j | (1 << b);
                    const R ar = re[j], ai = im[j], br = re[k], bi = im[k];
                    re[j] = ar + br;
                    im[j] = ai + bi;
                    re[k] = ar - br;
                    im[k] = ai - bi;
                }
            }
        }
    }
}

// Move the points from window layout a_old to window layout a_new through LDS.
template <typename R, int TL, int RL>
__device__ __forceinline__ void exchange(R (&re)[1 << RL], R (&im)[1 << RL], cx<R>* lds, int a_old, int a_new) {
    const uint32_t tid = threadIdx.x;
#pragma unroll
    for (int j = 0; j < (1 << RL); ++j) {
        cx<R> v;
        v.re = re[j];
        v.im = im[j];
        lds[padi(win_idx(tid, j, a_old, RL))] = v;
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < (1 << RL); ++j) {
        const cx<R> v = lds[padi(win_idx(tid, j, a_new, RL))];
        re[j] = v.re;
        im[j] = v.im;
    }
    __syncthreads();
}

// Unnormalised WHT over bits [lo_bit, K) of the tile index.  On entry thread t
// holds points t + j 2^TL (window a = TL); returns the window of the result.
template <typename R, int TL, int RL>
__device__ __forceinline__ int tile_fwht(R (&re)[1 << RL], R (&im)[1 << RL], cx<R>* lds, int lo_bit) {
    constexpr int K = TL + RL;
    int a = TL, hi = K;
    int lo = max(a, lo_bit);
    if (lo < hi) reg_stages<R, RL>(re, im, lo - a, hi - a);
    hi = lo;
    while (hi > lo_bit) {
        const int na = max(hi - RL, 0);
        exchange<R, TL, RL>(re, im, lds, a, na);
        a = na;
        lo = max(a, lo_bit);
        reg_stages<R, RL>(re, im, lo - a, hi - a);
        hi = lo;
    }
    return a;
}

// f values of the half-size problem at half indices (tile << K) + t + j 2^TL.
template <typename R, int TL, int RL>
__device__ __forceinline__ void load_products(const cx<R>* __restrict__ psi, int nh, uint32_t x, uint32_t tile,
                                              R (&re)[1 << RL], R (&im)[1 << RL]) {
    constexpr int K = TL + RL;
    const uint32_t tid = threadIdx.x;
    if (x != 0u) {
        const int p = 31 - __builtin_clz(x);
        const uint32_t lowmask = (1u << p) - 1u;
#pragma unroll
        for (int j = 0; j < (1 << RL); ++j) {
            const uint32_t bp = (tile << K) + tid + ((uint32_t)j << TL);
            const uint32_t b = (bp & lowmask) | ((bp & ~lowmask) << 1);
            const cx<R> a = psi[b];
            const cx<R> c = psi[b ^ x];
            re[j] = a.re * c.re + a.im * c.im;
            im[j] = a.re * c.im - a.im * c.re;
        }
    } else {
        const uint32_t half = 1u << nh;
#pragma unroll
        for (int j = 0; j < (1 << RL); ++j) {
            const uint32_t bp = (tile << K) + tid + ((uint32_t)j << TL);
            const cx<R> a = psi[bp];
            const cx<R> c = psi[bp + half];
            re[j] = a.re * a.re + a.im * a.im;
            im[j] = c.re * c.re + c.im * c.im;
        }
    }
}

// Per-thread accumulators in the transform precision, reduced in FP64.
// gap holds the largest |F|^2 below (1 - eps)^2 (-1 if none).
template <typename R>
struct Acc {
    R s1, ent, s2, s3, s4, gap;
    unsigned cnt;
    __device__ void init() { s1 = ent = s2 = s3 = s4 = R(0); gap = R(-1); cnt = 0u; }
};

struct AccD {
    double s1, ent, s2, s3, s4, gap;
    unsigned cnt;
};

template <typename R> struct Tiny;
template <> struct Tiny<float> { static constexpr float v = 1e-30f; };
template <> struct Tiny<double> { static constexpr double v = 1e-300; };

// One squared magnitude a2 = |F|^2 of the family: moments up to alpha = MOM,
// the Shannon term a2 log2 a2 (a2 below Tiny contributes below 1e-28), and the
// nullity test ||F| - 1| < eps written as (1-eps)^2 < a2 < (1+eps)^2.
template <typename R, int MOM>
__device__ __forceinline__ void acc_sq(Acc<R>& A, R a2, R lo2, R hi2) {
    A.s1 += a2;
    const R a4 = a2 * a2;
    A.s2 += a4;
    if constexpr (MOM >= 3) A.s3 = fma(a4, a2, A.s3);
    if constexpr (MOM >= 4) A.s4 = fma(a4, a4, A.s4);
    A.ent = fma(a2, Math<R>::lg2(fmax(a2, Tiny<R>::v)), A.ent);
    A.cnt += (a2 > lo2 && a2 < hi2) ? 1u : 0u;
    A.gap = fmax(A.gap, a2 <= lo2 ? a2 : R(-1));
}

// Both magnitudes carried by each point G of the half-size spectrum:
// x = 0: |Re G + Im G|, |Re G - Im G|;  x != 0: 2|Re G|, 2|Im G|.
template <typename R, int RL, int MOM>
__device__ __forceinline__ void acc_points(Acc<R>& A, const R (&re)[1 << RL], const R (&im)[1 << RL], bool x0, R lo2,
                                           R hi2) {
    if (x0) {
#pragma unroll
        for (int j = 0; j < (1 << RL); ++j) {
            const R u = re[j] + im[j], v = re[j] - im[j];
            acc_sq<R, MOM>(A, u * u, lo2, hi2);
            acc_sq<R, MOM>(A, v * v, lo2, hi2);
        }
    } else {
#pragma unroll
        for (int j = 0; j < (1 << RL); ++j) {
            const R u = re[j] + re[j], v = im[j] + im[j];
            acc_sq<R, MOM>(A, u * u, lo2, hi2);
            acc_sq<R, MOM>(A, v * v, lo2, hi2);
        }
    }
}

__device__ __forceinline__ void add_to(AccD& a, const AccD& b) {
    a.s1 += b.s1;
    a.ent += b.ent;
    a.s2 += b.s2;
    a.s3 += b.s3;
    a.s4 += b.s4;
    a.gap = fmax(a.gap, b.gap);
    a.cnt += b.cnt;
}

// Fixed-order reduction inside one wave (all lanes end with the same total).
template <int WS>
__device__ __forceinline__ AccD wave_reduce(AccD a) {
#pragma unroll
    for (int off = WS / 2; off > 0; off >>= 1) {
        a.s1 += __shfl_xor(a.s1, off);
        a.ent += __shfl_xor(a.ent, off);
        a.s2 += __shfl_xor(a.s2, off);
        a.s3 += __shfl_xor(a.s3, off);
        a.s4 += __shfl_xor(a.s4, off);
        a.gap = fmax(a.gap, __shfl_xor(a.gap, off));
        a.cnt += __shfl_xor(a.cnt, off);
    }
    return a;
}

// Fixed-order workgroup reduction; the total is valid in thread 0.
template <int NT>
__device__ AccD block_reduce(AccD a, AccD* sh) {
    a = wave_reduce<(NT < 64 ? NT : 64)>(a);
    if constexpr (NT > 64) {
        const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
        if (lane == 0) sh[wid] = a;
        __syncthreads();
        if (threadIdx.x == 0) {
            AccD t = sh[0];
            for (int w = 1; w < NT / 64; ++w) add_to(t, sh[w]);
            a = t;
        }
    }
    return a;
}

template <typename R>
__device__ __forceinline__ AccD widen(const Acc<R>& a) {
    AccD d;
    d.s1 = (double)a.s1;
    d.ent = (double)a.ent;
    d.s2 = (double)a.s2;
    d.s3 = (double)a.s3;
    d.s4 = (double)a.s4;
    d.gap = (double)a.gap;
    d.cnt = a.cnt;
    return d;
}

// Raw per-workgroup sums, stored in the FamilyRes layout.
__device__ __forceinline__ FamilyRes raw_res(const AccD& a, uint64_t x) {
    FamilyRes r;
    r.x = x;
    r.p = a.s1;
    r.ent = a.ent;
    r.m[0] = a.s2;
    r.m[1] = a.s3;
    r.m[2] = a.s4;
    r.gap = a.gap;
    r.nu = a.cnt;
    return r;
}

__device__ __forceinline__ AccD acc_of(const FamilyRes& r) {
    AccD a;
    a.s1 = r.p;
    a.ent = r.ent;
    a.s2 = r.m[0];
    a.s3 = r.m[1];
    a.s4 = r.m[2];
    a.gap = r.gap;
    a.cnt = (unsigned)r.nu;
    return a;
}

// Final per-family values: exact power-of-two scaling by d^-alpha (d = 2^n) and
// the gap as a magnitude.  Moments above MOM are reported as NaN (not computed).
template <int MOM>
__device__ __forceinline__ FamilyRes finish(const AccD& a, uint64_t x, int n) {
    FamilyRes r;
    r.x = x;
    r.p = ldexp(a.s1, -n);
    r.ent = a.ent;
    r.m[0] = ldexp(a.s2, -2 * n);
    r.m[1] = MOM >= 3 ? ldexp(a.s3, -3 * n) : __builtin_nan("");
    r.m[2] = MOM >= 4 ? ldexp(a.s4, -4 * n) : __builtin_nan("");
    r.gap = a.gap >= 0.0 ? sqrt(a.gap) : -1.0;
    r.nu = a.cnt;
    return r;
}

template <typename R>
__device__ __forceinline__ void thresholds(R eps, R& lo2, R& hi2) {
    lo2 = (R(1) - eps) * (R(1) - eps);
    hi2 = (R(1) + eps) * (R(1) + eps);
}

// ---------------------------------------------------------------------------
// Kernels
// ---------------------------------------------------------------------------

// Whole family in one workgroup (n - 1 = K).  Grid: one block per family.
template <typename R, int TL, int RL, int MOM>
__global__ void __launch_bounds__(1 << TL)
k_fused(const cx<R>* __restrict__ psi, int n, const uint64_t* __restrict__ xs, uint64_t x0, R eps,
        FamilyRes* __restrict__ out) {
    constexpr int K = TL + RL;
    constexpr int NT = 1 << TL;
    __shared__ cx<R> lds[Lds<K>::elems];
    __shared__ AccD shw[NT / 64 > 0 ? NT / 64 : 1];
    const uint32_t slot = blockIdx.x;
    const uint64_t x = xs ? xs[slot] : x0 + slot;
    R re[1 << RL], im[1 << RL];
    load_products<R, TL, RL>(psi, n - 1, (uint32_t)x, 0u, re, im);
    tile_fwht<R, TL, RL>(re, im, lds, 0);
    R lo2, hi2;
    thresholds(eps, lo2, hi2);
    Acc<R> acc;
    acc.init();
    acc_points<R, RL, MOM>(acc, re, im, x == 0, lo2, hi2);
    const AccD tot = block_reduce<NT>(widen(acc), shw);
    if (threadIdx.x == 0) out[slot] = finish<MOM>(tot, x, n);
}

// First pass of a multi-pass transform: products + low K index bits of one tile.
// Grid: (tiles per family, families).
template <typename R, int TL, int RL>
__global__ void __launch_bounds__(1 << TL)
k_first(const cx<R>* __restrict__ psi, int n, const uint64_t* __restrict__ xs, uint64_t x0,
        cx<R>* __restrict__ work) {
    constexpr int K = TL + RL;
    __shared__ cx<R> lds[Lds<K>::elems];
    const int nh = n - 1;
    const uint32_t tile = blockIdx.x, slot = blockIdx.y;
    const uint64_t x = xs ? xs[slot] : x0 + slot;
    R re[1 << RL], im[1 << RL];
    load_products<R, TL, RL>(psi, nh, (uint32_t)x, tile, re, im);
    const int a = tile_fwht<R, TL, RL>(re, im, lds, 0);
    cx<R>* dst = work + ((size_t)slot << nh) + ((size_t)tile << K);
#pragma unroll
    for (int j = 0; j < (1 << RL); ++j) {
        cx<R> v;
        v.re = re[j];
        v.im = im[j];
        dst[win_idx(threadIdx.x, j, a, RL)] = v;
    }
}

// Column pass over index bits [lo, lo + s) of every family in the batch.
// A tile is 2^s rows (stride 2^lo) by 2^w consecutive columns, w = K - s.
// Grid: (2^(nh - K), families).  LAST: reduce to one partial per workgroup
// (parts[family][block]) instead of writing the spectrum back.
template <typename R, int TL, int RL, bool LAST, int MOM>
__global__ void __launch_bounds__(1 << TL)
k_column(cx<R>* __restrict__ work, int n, int lo, int s, const uint64_t* __restrict__ xs, uint64_t x0, R eps,
         FamilyRes* __restrict__ parts) {
    constexpr int K = TL + RL;
    constexpr int NT = 1 << TL;
    __shared__ cx<R> lds[Lds<K>::elems];
    const int nh = n - 1;
    const int w = K - s;
    const int cbits = lo - w;
    const uint32_t bid = blockIdx.x, slot = blockIdx.y;
    const uint32_t cb = bid & ((1u << cbits) - 1u);
    const uint32_t hb = bid >> cbits;
    cx<R>* base = work + ((size_t)slot << nh) + ((size_t)hb << (lo + s)) + ((size_t)cb << w);
    const uint32_t wmask = (1u << w) - 1u;
    R re[1 << RL], im[1 << RL];
#pragma unroll
    for (int j = 0; j < (1 << RL); ++j) {
        const uint32_t i = threadIdx.x + ((uint32_t)j << TL);
        const cx<R> v = base[(i & wmask) + ((size_t)(i >> w) << lo)];
        re[j] = v.re;
        im[j] = v.im;
    }
    const int a = tile_fwht<R, TL, RL>(re, im, lds, w);
    if constexpr (!LAST) {
#pragma unroll
        for (int j = 0; j < (1 << RL); ++j) {
            const uint32_t i = win_idx(threadIdx.x, j, a, RL);
            cx<R> v;
            v.re = re[j];
            v.im = im[j];
            base[(i & wmask) + ((size_t)(i >> w) << lo)] = v;
        }
    } else {
        __shared__ AccD shw[NT / 64 > 0 ? NT / 64 : 1];
        const uint64_t x = xs ? xs[slot] : x0 + slot;
        R lo2, hi2;
        thresholds(eps, lo2, hi2);
        Acc<R> acc;
        acc.init();
        acc_points<R, RL, MOM>(acc, re, im, x == 0, lo2, hi2);
        const AccD tot = block_reduce<NT>(widen(acc), shw);
        if (threadIdx.x == 0) parts[(size_t)slot * gridDim.x + bid] = raw_res(tot, x);
    }
}

// Per-family fixed-order sum of the final pass's partials.  Grid: one wave per family.
template <int MOM>
__global__ void __launch_bounds__(64)
k_finalize(const FamilyRes* __restrict__ parts, int nblk, int n, FamilyRes* __restrict__ out) {
    const FamilyRes* p = parts + (size_t)blockIdx.x * nblk;
    AccD a;
    a.s1 = a.ent = a.s2 = a.s3 = a.s4 = 0.0;
    a.gap = -1.0;
    a.cnt = 0u;
    for (int i = threadIdx.x; i < nblk; i += 64) add_to(a, acc_of(p[i]));
    a = wave_reduce<64>(a);
    if (threadIdx.x == 0) out[blockIdx.x] = finish<MOM>(a, p[0].x, n);
}

// Fixed-order sum of count per-family results into one SweepSums.
__global__ void __launch_bounds__(256)
k_reduce_fam(const FamilyRes* __restrict__ in, int64_t count, SweepSums* __restrict__ out) {
    constexpr int NT = 256;
    __shared__ SweepSums sh[NT];
    SweepSums t;
    t.S[0] = t.S[1] = t.S[2] = t.L = t.P = 0.0;
    t.gap = -1.0;
    t.nu_cnt = 0;
    t.count = 0;
    for (int64_t i = threadIdx.x; i < count; i += NT) {
        const FamilyRes v = in[i];
        t.S[0] += v.m[0];
        t.S[1] += v.m[1];
        t.S[2] += v.m[2];
        t.L += v.ent;
        t.P += v.p;
        t.gap = fmax(t.gap, v.gap);
        t.nu_cnt += v.nu;
        t.count += 1;
    }
    sh[threadIdx.x] = t;
    __syncthreads();
    for (int h = NT / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) {
            SweepSums& a = sh[threadIdx.x];
            const SweepSums& b = sh[threadIdx.x + h];
            a.S[0] += b.S[0];
            a.S[1] += b.S[1];
            a.S[2] += b.S[2];
            a.L += b.L;
            a.P += b.P;
            a.gap = fmax(a.gap, b.gap);
            a.nu_cnt += b.nu_cnt;
            a.count += b.count;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = sh[0];
}

// c(x, z) = (-i)^{|x&z|} F_x(z) from the half spectrum G of one family.
template <typename R>
__global__ void k_signed(const cx<R>* __restrict__ G, int n, uint32_t x, double* __restrict__ c) {
    const uint64_t d = 1ull << n;
    const uint64_t z = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (z >= d) return;
    const int nh = n - 1;
    double v;
    if (x == 0u) {
        const cx<R> g = G[z & ((1ull << nh) - 1ull)];
        v = ((z >> nh) & 1ull) ? (double)g.re - (double)g.im : (double)g.re + (double)g.im;
    } else {
        const int p = 31 - __builtin_clz(x);
        const uint64_t lowmask = (1ull << p) - 1ull;
        const uint64_t zp = (z & lowmask) | ((z >> (p + 1)) << p);
        const cx<R> g = G[zp];
        const int k = __popcll((uint64_t)x & z);
        if (k & 1) v = ((k >> 1) & 1 ? -2.0 : 2.0) * (double)g.im;
        else v = ((k >> 1) & 1 ? -2.0 : 2.0) * (double)g.re;
    }
    c[z] = v;
}

__global__ void __launch_bounds__(256)
k_reduce_sweep(const SweepSums* __restrict__ in, int64_t count, SweepSums* __restrict__ out) {
    constexpr int NT = 256;
    __shared__ SweepSums sh[NT];
    SweepSums t;
    t.S[0] = t.S[1] = t.S[2] = t.L = t.P = 0.0;
    t.gap = -1.0;
    t.nu_cnt = 0;
    t.count = 0;
    for (int64_t i = threadIdx.x; i < count; i += NT) {
        const SweepSums v = in[i];
        t.S[0] += v.S[0];
        t.S[1] += v.S[1];
        t.S[2] += v.S[2];
        t.L += v.L;
        t.P += v.P;
        t.gap = fmax(t.gap, v.gap);
        t.nu_cnt += v.nu_cnt;
        t.count += v.count;
    }
    sh[threadIdx.x] = t;
    __syncthreads();
    for (int h = NT / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) {
            SweepSums& a = sh[threadIdx.x];
            const SweepSums& b = sh[threadIdx.x + h];
            a.S[0] += b.S[0];
            a.S[1] += b.S[1];
            a.S[2] += b.S[2];
            a.L += b.L;
            a.P += b.P;
            a.gap = fmax(a.gap, b.gap);
            a.nu_cnt += b.nu_cnt;
            a.count += b.count;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = sh[0];
}

// Tile shapes: first pass K = 12 (256 threads x 16 points); column passes K = 13
// single (512 x 16) / 12 double (256 x 16); fused kernels K = n - 1.
constexpr int K_FIRST = 12;
template <typename R> struct ColShape;
template <> struct ColShape<float> { static constexpr int TL = 9, RL = 4; };
template <> struct ColShape<double> { static constexpr int TL = 8, RL = 4; };

template <typename R, int K, int MOM>
hipError_t launch_fused_k(const void* psi, int n, const uint64_t* xs, uint64_t x0, int nb, R eps, FamilyRes* out,
                          hipStream_t st) {
    constexpr int RL0 = K < 4 ? K : 4;
    constexpr int TL = K == 13 ? 9 : K - RL0;
    constexpr int RL = K - TL;
    hipLaunchKernelGGL((k_fused<R, TL, RL, MOM>), dim3(nb), dim3(1 << TL), 0, st, (const cx<R>*)psi, n, xs, x0, eps,
                       out);
    return hipGetLastError();
}

template <typename R, int MOM>
hipError_t launch_fused(const void* psi, int n, const uint64_t* xs, uint64_t x0, int nb, R eps, FamilyRes* out,
                        hipStream_t st) {
    switch (n - 1) {
#define PW_CASE(K) \
    case K: return launch_fused_k<R, K, MOM>(psi, n, xs, x0, nb, eps, out, st);
        PW_CASE(0) PW_CASE(1) PW_CASE(2) PW_CASE(3) PW_CASE(4) PW_CASE(5) PW_CASE(6)
        PW_CASE(7) PW_CASE(8) PW_CASE(9) PW_CASE(10) PW_CASE(11) PW_CASE(12)
#undef PW_CASE
        case 13:
            if constexpr (sizeof(R) == 4) return launch_fused_k<R, 13, MOM>(psi, n, xs, x0, nb, eps, out, st);
            return hipErrorInvalidValue;
        default: return hipErrorInvalidValue;
    }
}

template <typename R, int MOM>
hipError_t eval_batch_t(const Plan& P, const void* psi, const uint64_t* xs, uint64_t x0, int nb, double eps,
                        void* work, FamilyRes* parts, FamilyRes* out, hipStream_t st, const LaunchTimer* tm) {
    if (nb <= 0) return hipSuccess;
    const R e = (R)eps;
    if (P.fused) {
        if (tm) tm->begin(tm->self, 0, st);
        hipError_t err = launch_fused<R, MOM>(psi, P.n, xs, x0, nb, e, out, st);
        if (tm) tm->end(tm->self, 0, nb, st);
        return err;
    }
    constexpr int TL = ColShape<R>::TL, RL = ColShape<R>::RL;
    if (tm) tm->begin(tm->self, 1, st);
    hipLaunchKernelGGL((k_first<R, 8, 4>), dim3(1u << (P.nh - K_FIRST), nb), dim3(256), 0, st, (const cx<R>*)psi,
                       P.n, xs, x0, (cx<R>*)work);
    if (tm) tm->end(tm->self, 1, nb, st);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
    const dim3 grid(1u << (P.nh - (TL + RL)), nb);
    for (int i = 0; i < P.npass; ++i) {
        const bool last = i + 1 == P.npass;
        if (tm) tm->begin(tm->self, last ? 3 : 2, st);
        if (!last) {
            hipLaunchKernelGGL((k_column<R, TL, RL, false, MOM>), grid, dim3(1 << TL), 0, st, (cx<R>*)work, P.n,
                               P.lo[i], P.s[i], xs, x0, e, parts);
        } else {
            hipLaunchKernelGGL((k_column<R, TL, RL, true, MOM>), grid, dim3(1 << TL), 0, st, (cx<R>*)work, P.n,
                               P.lo[i], P.s[i], xs, x0, e, parts);
        }
        if (tm) tm->end(tm->self, last ? 3 : 2, nb, st);
        err = hipGetLastError();
        if (err != hipSuccess) return err;
    }
    hipLaunchKernelGGL((k_finalize<MOM>), dim3(nb), dim3(64), 0, st, parts, (int)grid.x, P.n, out);
    return hipGetLastError();
}

template <typename R>
hipError_t transform_one_t(const Plan& P, const void* psi, uint64_t x, void* work, hipStream_t st) {
    // the multi-pass schedule without the final reduction
    constexpr int TL = ColShape<R>::TL, RL = ColShape<R>::RL;
    const int nh = P.nh;
    if (P.fused || nh <= K_FIRST) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_first<R, 8, 4>), dim3(1u << (nh - K_FIRST), 1), dim3(256), 0, st, (const cx<R>*)psi, P.n,
                       (const uint64_t*)nullptr, x, (cx<R>*)work);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
    for (int i = 0; i < P.npass; ++i) {
        hipLaunchKernelGGL((k_column<R, TL, RL, false, 2>), dim3(1u << (nh - (TL + RL)), 1), dim3(1 << TL), 0, st,
                           (cx<R>*)work, P.n, P.lo[i], P.s[i], (const uint64_t*)nullptr, x, (R)0,
                           (FamilyRes*)nullptr);
        err = hipGetLastError();
        if (err != hipSuccess) return err;
    }
    return hipSuccess;
}

}  // namespace

Plan make_plan(int n, bool dbl) {
    Plan P{};
    P.n = n;
    P.nh = n - 1;
    const int fmax = dbl ? 12 : 13;
    const int ktile = dbl ? 12 : 13;
    const int smax = dbl ? 9 : 9;  // keeps columns >= 128 bytes
    if (P.nh <= fmax) {
        P.fused = true;
        P.k1 = P.nh;
        P.npass = 0;
        P.blocks_last = 1;
        return P;
    }
    P.fused = false;
    P.k1 = K_FIRST;
    const int rem = P.nh - K_FIRST;
    const int np = (rem + smax - 1) / smax;
    P.npass = np;
    int lo = K_FIRST;
    for (int i = 0; i < np; ++i) {
        const int left = P.nh - lo;
        const int s = (left + (np - i) - 1) / (np - i);  // balanced split, largest first
        P.lo[i] = lo;
        P.s[i] = s;
        lo += s;
    }
    P.blocks_last = 1 << (P.nh - ktile);
    return P;
}

hipError_t eval_batch(const Plan& P, bool dbl, int max_alpha, const void* psi, const uint64_t* xs, uint64_t x0,
                      int nb, double eps, void* work, FamilyRes* parts, FamilyRes* out, hipStream_t st,
                      const LaunchTimer* tm) {
    if (dbl)
        return max_alpha >= 4 ? eval_batch_t<double, 4>(P, psi, xs, x0, nb, eps, work, parts, out, st, tm)
                              : eval_batch_t<double, 2>(P, psi, xs, x0, nb, eps, work, parts, out, st, tm);
    return max_alpha >= 4 ? eval_batch_t<float, 4>(P, psi, xs, x0, nb, eps, work, parts, out, st, tm)
                          : eval_batch_t<float, 2>(P, psi, xs, x0, nb, eps, work, parts, out, st, tm);
}

hipError_t reduce_families(const FamilyRes* in, int64_t count, SweepSums* out, hipStream_t st) {
    hipLaunchKernelGGL(k_reduce_fam, dim3(1), dim3(256), 0, st, in, count, out);
    return hipGetLastError();
}

hipError_t transform_one(const Plan& P, bool dbl, const void* psi, uint64_t x, void* work, hipStream_t st) {
    return dbl ? transform_one_t<double>(P, psi, x, work, st) : transform_one_t<float>(P, psi, x, work, st);
}

hipError_t signed_values(const Plan& P, bool dbl, const void* G, uint64_t x, double* c, hipStream_t st) {
    const uint64_t d = 1ull << P.n;
    const dim3 grid((unsigned)((d + 255) / 256));
    if (dbl)
        hipLaunchKernelGGL(k_signed<double>, grid, dim3(256), 0, st, (const cx<double>*)G, P.n, (uint32_t)x, c);
    else
        hipLaunchKernelGGL(k_signed<float>, grid, dim3(256), 0, st, (const cx<float>*)G, P.n, (uint32_t)x, c);
    return hipGetLastError();
}

hipError_t reduce_sweep(const SweepSums* in, int64_t count, SweepSums* out, hipStream_t st) {
    hipLaunchKernelGGL(k_reduce_sweep, dim3(1), dim3(256), 0, st, in, count, out);
    return hipGetLastError();
}

}  // namespace pw
