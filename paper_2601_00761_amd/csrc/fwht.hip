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
// registers.  The sequence of register windows is fixed at compile time, so
// every LDS and global address is a per-thread base plus an immediate offset.
// Small states (n - 1 <= 13 single / 12 double) run the whole transform and the
// reductions in one workgroup per family.  Larger states use a first pass over
// the low 12 index bits (contiguous tiles, products formed at load time) and
// column passes over the remaining bits (tiles of 2^s rows by 2^w >= 128-byte
// columns); the last column pass reduces in registers and never writes the
// spectrum back.  Per-workgroup FP64 partials are summed per family in a fixed
// order by a separate finalize kernel, so results are bitwise reproducible.
#include "common.h"
#include <hip/hip_ext.h>
#include <math.h>

namespace pw {
namespace {

template <typename R> struct Math;
template <> struct Math<float> {
    static __device__ __forceinline__ float lg2(float v) { return __log2f(v); }
    static constexpr float tiny = 1e-30f;
};
template <> struct Math<double> {
    // log2 of a positive double (here >= 1e-300) by the inverse hyperbolic tangent
    // series: v = m 2^e with m in [sqrt(1/2), sqrt(2)), ln m = 2 atanh(s) with
    // s = (m - 1) / (m + 1), |s| <= 0.1716, and atanh s = s (1 + s^2/3 + s^4/5 + ...);
    // the terms through s^21 leave a truncation below 2^-54 relative.  m - 1 is exact.
    // About a third of the instructions of the library log2, at a few ulp.
    static __device__ __forceinline__ double lg2(double v) {
        int e;
        double m = __builtin_frexp(v, &e);  // m in [1/2, 1)
        if (m < 0.70710678118654752) {
            m *= 2.0;
            e -= 1;
        }
        // s = (m - 1) / (m + 1) with the hardware reciprocal refined by two Newton steps
        // (the denominator lies in [1.7, 2.5]; error a few ulp, well inside the series' use)
        const double den = m + 1.0;
        double rc = __builtin_amdgcn_rcp(den);
        rc = fma(fma(-den, rc, 1.0), rc, rc);
        rc = fma(fma(-den, rc, 1.0), rc, rc);
        const double num = m - 1.0;
        double s = num * rc;
        s = fma(fma(-den, s, num), rc, s);
        const double s2 = s * s;
        double p = 1.0 / 21.0;
        p = fma(p, s2, 1.0 / 19.0);
        p = fma(p, s2, 1.0 / 17.0);
        p = fma(p, s2, 1.0 / 15.0);
        p = fma(p, s2, 1.0 / 13.0);
        p = fma(p, s2, 1.0 / 11.0);
        p = fma(p, s2, 1.0 / 9.0);
        p = fma(p, s2, 1.0 / 7.0);
        p = fma(p, s2, 1.0 / 5.0);
        p = fma(p, s2, 1.0 / 3.0);
        const double at = fma(s * s2, p, s);
        constexpr double two_over_ln2 = 2.8853900817779268;  // 2 / ln 2
        return fma(at, two_over_ln2, (double)e);
    }
    static constexpr double tiny = 1e-300;
};

// FP64 log2 for the reductions by a 256-entry table: v = 2^e m, m in [1, 2), c = 1 + i/256
// with i the top 8 fraction bits of m (so m - c is exact and 0 <= r = (m - c)/c < 2^-8),
// log2 v = e + log2 c + log2(1 + r), the last by its series through r^6 (truncation below
// r^7 / (7 ln 2) < 2^-58).  For m >= 1.5 the entry holds log2(c / 2) and e counts one more,
// so that v just below a power of two does not lose its small logarithm to cancellation.
// A few ulp (checked against 120-bit logarithms over 1e-300 .. 3; absolute error below
// 4e-18 within 1 % of 1).  Each workgroup fills its table once (1/c by IEEE division,
// log2 by the series above); a lookup then costs about ten FP64 operations against some
// twenty-five for the series alone.
struct Lg2Entry {
    double inv, lg;   // 1 / c_i, log2 c_i (log2(c_i / 2) for i >= 128)
};
constexpr int LG2_TAB = 256;

// All threads of the workgroup call this (it ends with a barrier).
__device__ __forceinline__ void lg2_table_init(Lg2Entry* tab) {
    for (int i = threadIdx.x; i < LG2_TAB; i += blockDim.x) {
        const double c = 1.0 + (double)i / LG2_TAB;
        tab[i].inv = 1.0 / c;
        tab[i].lg = Math<double>::lg2(i >= LG2_TAB / 2 ? 0.5 * c : c);
    }
    __syncthreads();
}

__device__ __forceinline__ double lg2_tab(double v, const Lg2Entry* tab) {
    const uint64_t bits = (uint64_t)__double_as_longlong(v);
    const uint32_t hi = (uint32_t)(bits >> 32);
    const uint32_t i = (hi >> 12) & (LG2_TAB - 1u);
    const int e = (int)(hi >> 20) - 1023 + (int)(i >> 7);   // v is a positive normal number
    const double m = __longlong_as_double((long long)((bits & 0x000FFFFFFFFFFFFFull) | 0x3FF0000000000000ull));
    const double c = __longlong_as_double((long long)(0x3FF0000000000000ull | ((uint64_t)i << 44)));
    const Lg2Entry t = tab[i];
    const double r = (m - c) * t.inv;
    constexpr double L = 1.4426950408889634;   // 1 / ln 2
    double p = -L / 6.0;
    p = fma(p, r, L / 5.0);
    p = fma(p, r, -L / 4.0);
    p = fma(p, r, L / 3.0);
    p = fma(p, r, -L / 2.0);
    p = fma(p, r, L);
    return ((double)e + t.lg) + r * p;
}

// log2 in the reductions: the hardware FP32 instruction, or the FP64 table.
template <typename R>
__device__ __forceinline__ R red_lg2(R v, const Lg2Entry* tab) {
    if constexpr (sizeof(R) == 4) return Math<float>::lg2(v);
    else return lg2_tab(v, tab);
}

// The table a kernel needs for its reductions: one per workgroup for FP64, none for FP32.
template <typename R> struct Lg2Shared {
    static constexpr int n = sizeof(R) == 8 ? LG2_TAB : 1;
};

// Window layout: register bits [A, A + RL) of the tile index, thread bits the rest.
template <int A, int RL>
__device__ __forceinline__ uint32_t thread_part(uint32_t tid) {
    return (tid & ((1u << A) - 1u)) | ((tid >> A) << (A + RL));
}
__host__ __device__ constexpr uint32_t padc(uint32_t i) { return i + (i >> 4); }
__device__ __forceinline__ uint32_t padi(uint32_t i) { return i + (i >> 4); }

template <int K> struct Lds { static constexpr int elems = (1 << K) + ((1 << K) >> 4); };

// The butterflies of reg_stages (below) over register bits [B0, B1), taken depth first:
// the 2^M registers from OFF are finished over their own bits below M - 1 before the
// stage on bit M - 1 joins the two halves.  Each point still takes its bits from low to
// high and each butterfly sees the operands it sees in the stage-by-stage order, so the
// results are identical; but the stages of the registers loaded first can run while the
// later loads are still in flight.  DepthFirst1 takes one array of parts (real or
// imaginary), DepthFirst both parts of each point together.
template <typename R, int RL, int B0, int B1, int OFF, int M>
struct DepthFirst1 {
    static __device__ __forceinline__ void run(R (&v)[1 << RL]) {
        if constexpr (M > 0) {
            DepthFirst1<R, RL, B0, B1, OFF, M - 1>::run(v);
            DepthFirst1<R, RL, B0, B1, OFF + (1 << (M - 1)), M - 1>::run(v);
            constexpr int b = M - 1;
            if constexpr (b >= B0 && b < B1) {
#pragma unroll
                for (int i = 0; i < (1 << b); ++i) {
                    const int j = OFF + i, k = j + (1 << b);
                    const R a = v[j], c = v[k];
                    v[j] = a + c;
                    v[k] = a - c;
                }
            }
        }
    }
};

template <typename R, int RL, int B0, int B1, int OFF, int M>
struct DepthFirst {
    static __device__ __forceinline__ void run(R (&re)[1 << RL], R (&im)[1 << RL]) {
        if constexpr (M > 0) {
            DepthFirst<R, RL, B0, B1, OFF, M - 1>::run(re, im);
            DepthFirst<R, RL, B0, B1, OFF + (1 << (M - 1)), M - 1>::run(re, im);
            constexpr int b = M - 1;
            if constexpr (b >= B0 && b < B1) {
#pragma unroll
                for (int i = 0; i < (1 << b); ++i) {
                    const int j = OFF + i, k = j + (1 << b);
                    const R ar = re[j], ai = im[j], br = re[k], bi = im[k];
                    re[j] = ar + br;
                    im[j] = ai + bi;
                    re[k] = ar - br;
                    im[k] = ai - bi;
                }
            }
        }
    }
};

// Radix-2 butterflies (u, v) -> (u + v, u - v) over register bits [B0, B1).
template <typename R, int RL, int B0, int B1>
__device__ __forceinline__ void reg_stages(R (&re)[1 << RL], R (&im)[1 << RL]) {
#pragma unroll
    for (int b = B0; b < B1; ++b) {
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

// Move the points from window AO to window AN through LDS.  The address of
// (thread t, register j) in window A is pad(T_A(t) | j 2^A) = pad(T_A(t)) + pad(j 2^A)
// (the two parts have disjoint bits), i.e. a per-thread base plus a constant.
// TRAIL: end with a barrier, needed only when the same buffer is written again
// before every thread has passed another barrier.
template <typename R, int TL, int RL, int AO, int AN, bool TRAIL = true>
__device__ __forceinline__ void exchange(R (&re)[1 << RL], R (&im)[1 << RL], cx<R>* lds) {
    const uint32_t tid = threadIdx.x;
    cx<R>* wo = lds + padi(thread_part<AO, RL>(tid));
#pragma unroll
    for (int j = 0; j < (1 << RL); ++j) {
        cx<R> v;
        v.re = re[j];
        v.im = im[j];
        wo[padc((uint32_t)j << AO)] = v;
    }
    __syncthreads();
    const cx<R>* rn = lds + padi(thread_part<AN, RL>(tid));
#pragma unroll
    for (int j = 0; j < (1 << RL); ++j) {
        const cx<R> v = rn[padc((uint32_t)j << AN)];
        re[j] = v.re;
        im[j] = v.im;
    }
    if constexpr (TRAIL) __syncthreads();
}

// The same move for tiles too large for one complex LDS buffer (2^15 single-
// precision points = 256 KB > 160 KB): real parts first, then imaginary parts,
// through a float buffer padded one element in 2^RL.  A thread part that strides
// 2^(A + RL) between groups of 2^A lanes then lands each group on its own bank range
// (64 banks; RL = 5 or 6 with A = 3 gives 8 groups of 8 lanes, RL = 5 with A = 0
// one lane per bank).
template <int RL>
__host__ __device__ constexpr uint32_t pads(uint32_t i) { return i + (i >> RL); }

// An empty statement that reads and writes every element: the arithmetic before it stays
// before it (the compiler otherwise sinks the butterflies below the next barrier).
template <typename R, int RL>
__device__ __forceinline__ void settle(R (&v)[1 << RL]) {
#pragma unroll
    for (int j = 0; j < (1 << RL); ++j) asm volatile("" : "+v"(v[j]));
}

// NB > 0: each part, as soon as it is back in registers, takes its butterflies over
// register bits [0, NB) depth first (the real parts' while the imaginary parts wait for
// the buffer): the same operations as the stages after the move, in another order.
template <typename R, int TL, int RL, int AO, int AN, bool TRAIL = true, int NB = 0>
__device__ __forceinline__ void exchange_split(R (&re)[1 << RL], R (&im)[1 << RL], R* buf) {
    static_assert(RL >= 4, "the split buffer pads one element in 2^min(RL, 5)");
    const uint32_t tid = threadIdx.x;
    R* wo = buf + pads<RL>(thread_part<AO, RL>(tid));
    const R* rn = buf + pads<RL>(thread_part<AN, RL>(tid));
#pragma unroll
    for (int j = 0; j < (1 << RL); ++j) wo[pads<RL>((uint32_t)j << AO)] = re[j];
    __syncthreads();
#pragma unroll
    for (int j = 0; j < (1 << RL); ++j) re[j] = rn[pads<RL>((uint32_t)j << AN)];
    if constexpr (NB > 0) {
        DepthFirst1<R, RL, 0, NB, 0, RL>::run(re);
        settle<R, RL>(re);
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < (1 << RL); ++j) wo[pads<RL>((uint32_t)j << AO)] = im[j];
    __syncthreads();
#pragma unroll
    for (int j = 0; j < (1 << RL); ++j) im[j] = rn[pads<RL>((uint32_t)j << AN)];
    if constexpr (NB > 0) DepthFirst1<R, RL, 0, NB, 0, RL>::run(im);
    if constexpr (TRAIL) __syncthreads();
}

// LDS bytes of a tile of 2^K points (split buffers pad one element per 2^min(RL, 5)).
template <typename R, int K, bool SPLIT, int RL>
struct LdsBytes {
    static constexpr size_t v = SPLIT ? ((size_t)(1 << K) + ((1 << K) >> (RL < 5 ? RL : 5))) * sizeof(R)
                                      : ((size_t)(1 << K) + ((1 << K) >> 4)) * sizeof(cx<R>);
};

// After the first round (window TL, register bits [max(TL, LO), K)), the bits
// [LO, TL) are taken in blocks of RL from the bottom: window B0 transforms
// [B0, min(B0 + RL, TL)).  The result stays in the last window, whose low
// threads hold consecutive indices (coalesced stores).
template <int TL, int RL, int LO>
constexpr int final_window() {
    if (LO >= TL) return TL;
    int b0 = LO;
    while (b0 + RL < TL) b0 += RL;
    return b0;
}

// REUSE: the workgroup runs another transform through the same buffer afterwards, so
// every exchange closes with a barrier; otherwise the last one needs none.
// DF: register stages depth first, on a split move each part's as it arrives.
template <typename R, int TL, int RL, int A, int B0, bool SPLIT, bool REUSE, bool DF = false>
struct Rounds {
    static __device__ __forceinline__ void run(R (&re)[1 << RL], R (&im)[1 << RL], void* lds) {
        if constexpr (B0 < TL) {
            constexpr bool trail = REUSE || B0 + RL < TL;
            constexpr int B1 = (B0 + RL < TL) ? B0 + RL : TL;
            if constexpr (SPLIT && DF) {
                exchange_split<R, TL, RL, A, B0, trail, B1 - B0>(re, im, (R*)lds);
            } else {
                if constexpr (SPLIT) exchange_split<R, TL, RL, A, B0, trail>(re, im, (R*)lds);
                else exchange<R, TL, RL, A, B0, trail>(re, im, (cx<R>*)lds);
                if constexpr (DF) DepthFirst<R, RL, 0, B1 - B0, 0, RL>::run(re, im);
                else reg_stages<R, RL, 0, B1 - B0>(re, im);
            }
            Rounds<R, TL, RL, B0, B0 + RL, SPLIT, REUSE, DF>::run(re, im, lds);
        }
    }
};

// Unnormalised WHT over bits [LO, K) of the tile index.  On entry thread t holds
// points t + j 2^TL (window TL); on exit the points are in final_window().
// DF: register stages depth first, starting while the loads are still in flight
// (the column passes: one workgroup per CU, so only the workgroup itself can fill the
// wait for its loads and its LDS moves).
template <typename R, int TL, int RL, int LO, bool SPLIT = false, bool REUSE = false, bool DF = false>
__device__ __forceinline__ void tile_fwht(R (&re)[1 << RL], R (&im)[1 << RL], void* lds) {
    constexpr int S0 = LO > TL ? LO : TL;
    if constexpr (DF) DepthFirst<R, RL, S0 - TL, RL, 0, RL>::run(re, im);
    else reg_stages<R, RL, S0 - TL, RL>(re, im);
    Rounds<R, TL, RL, TL, LO, SPLIT, REUSE, DF>::run(re, im, lds);
}

// f values of the half-size problem at half indices (tile << K) + t + j 2^TL
// (general x; used by the single-workgroup kernel and for x < 2^K).
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
        const cx<R>* pa = psi + (tile << K) + tid;
        const cx<R>* pc = pa + half;
#pragma unroll
        for (int j = 0; j < (1 << RL); ++j) {
            const cx<R> a = pa[(uint32_t)j << TL];
            const cx<R> c = pc[(uint32_t)j << TL];
            re[j] = a.re * a.re + a.im * a.im;
            im[j] = c.re * c.re + c.im * c.im;
        }
    }
}

// Same for x >= 2^K: the top bit p >= K only moves the tile, so the state
// tile is tu << K and the partner tile (tu ^ (x >> K)) << K, read at l ^ (x mod 2^K).
template <typename R, int TL, int RL>
__device__ __forceinline__ void load_products_hi(const cx<R>* __restrict__ psi, uint32_t x, uint32_t tile,
                                                 R (&re)[1 << RL], R (&im)[1 << RL]) {
    constexpr int K = TL + RL;
    const uint32_t tid = threadIdx.x;
    const uint32_t xh = x >> K, xl = x & ((1u << K) - 1u);
    const int q = 31 - __builtin_clz(xh);
    const uint32_t lowm = (1u << q) - 1u;
    const uint32_t tu = (tile & lowm) | ((tile & ~lowm) << 1);
    const cx<R>* pa = psi + ((size_t)tu << K) + tid;
    const cx<R>* pc = psi + ((size_t)(tu ^ xh) << K) + (tid ^ (xl & ((1u << TL) - 1u)));
    const uint32_t jx = xl >> TL;
#pragma unroll
    for (int j = 0; j < (1 << RL); ++j) {
        const cx<R> a = pa[(uint32_t)j << TL];
        const cx<R> c = pc[((uint32_t)j ^ jx) << TL];
        re[j] = a.re * c.re + a.im * c.im;
        im[j] = a.re * c.im - a.im * c.re;
    }
}

// Mixed states (Supplemental Material, mixed states): for Paulis supported on the
// first n_a qubits the family of x_A is the n_a-bit WHT of
//     h(a) = sum_e conj(psi(a, e)) psi(a ^ x_A, e) = rho_A[a ^ x_A, a],
// rho_A = Psi Psi^dagger the reduced density matrix.  It is stored family by family,
// D[x_A][a] = rho_A[a ^ x_A, a] (d_A x d_A, row x_A is the h of family x_A), so that a
// family reads one contiguous row.  h has the same Hermitian symmetry as f_x, so the
// half-size transform applies unchanged.
// h values of tile `tile` (half indices (tile << K) + t + j 2^TL) of family x.
template <typename R, int TL, int RL>
__device__ __forceinline__ void load_reduced(const cx<R>* __restrict__ D, int na, uint32_t x, uint32_t tile,
                                             R (&re)[1 << RL], R (&im)[1 << RL]) {
    constexpr int K = TL + RL;
    const uint32_t tid = threadIdx.x;
    const size_t dA = (size_t)1 << na;
    const cx<R>* row = D + (size_t)x * dA;
    if (x != 0u) {
        const int p = 31 - __builtin_clz(x);
        const uint32_t lowmask = (1u << p) - 1u;
#pragma unroll
        for (int j = 0; j < (1 << RL); ++j) {
            const uint32_t bp = (tile << K) + tid + ((uint32_t)j << TL);
            const uint32_t b = (bp & lowmask) | ((bp & ~lowmask) << 1);
            const cx<R> v = row[b];
            re[j] = v.re;
            im[j] = v.im;
        }
    } else {
        // h_0(a) = rho_A[a, a] is real: the two halves of a packed as re / im
        const uint32_t half = (uint32_t)(dA >> 1);
#pragma unroll
        for (int j = 0; j < (1 << RL); ++j) {
            const uint32_t bp = (tile << K) + tid + ((uint32_t)j << TL);
            re[j] = row[bp].re;
            im[j] = row[bp + half].re;
        }
    }
}

struct AccD {
    double s1, ent, s2, s3, s4, gap;
    unsigned cnt;
};

// The state a family reads: one state for the launch, or (lists over several states of
// one size) fpsi[slot], the device address of that family's state.
template <typename T>
__device__ __forceinline__ const T* state_of(const T* psi, const uint64_t* __restrict__ fpsi, uint32_t slot) {
    return fpsi ? reinterpret_cast<const T*>(fpsi[slot]) : psi;
}

// Reductions over the thread's points.  Each point carries two magnitudes:
// x = 0: |Re G + Im G|, |Re G - Im G|;  x != 0: 2|Re G|, 2|Im G|.  For x != 0 the
// squares are accumulated as t = (Re G)^2 and scaled by the exact factor 4 at the
// end (|F|^2 log2 |F|^2 = 4 t log2 t + 8 t).  Per square: moments up to MOM, the
// Shannon term (values below Math::tiny contribute < 1e-28) and the running
// maximum.  The nullity test (1-eps)^2 < |F|^2 < (1+eps)^2 and the gap (largest
// |F|^2 below (1-eps)^2) only need a second look when the maximum exceeds
// (1-eps)^2, which is rare outside stabilizer-like families.
template <typename R, int RL, int MOM>
__device__ __forceinline__ AccD reduce_points(const R (&re)[1 << RL], const R (&im)[1 << RL], bool x0, R eps,
                                              const Lg2Entry* tab) {
    // transform-precision partial sums over at most 16 points (32 magnitudes), then FP64
    constexpr int CH = (1 << RL) < 16 ? (1 << RL) : 16;
    double D1, D2, D3, D4, DE;
    R mx = R(0);
#pragma unroll
    for (int c0 = 0; c0 < (1 << RL); c0 += CH) {
        R s1 = R(0), s2 = R(0), s3 = R(0), s4 = R(0), ent = R(0);
        auto acc = [&](R t) {
            s1 += t;
            const R t2 = t * t;
            s2 += t2;
            if constexpr (MOM >= 3) s3 = fma(t2, t, s3);
            if constexpr (MOM >= 4) s4 = fma(t2, t2, s4);
            ent = fma(t, red_lg2<R>(fmax(t, Math<R>::tiny), tab), ent);
            mx = fmax(mx, t);
        };
        if (x0) {
#pragma unroll
            for (int j = c0; j < c0 + CH; ++j) {
                const R u = re[j] + im[j], v = re[j] - im[j];
                acc(u * u);
                acc(v * v);
            }
        } else {
#pragma unroll
            for (int j = c0; j < c0 + CH; ++j) {
                acc(re[j] * re[j]);
                acc(im[j] * im[j]);
            }
        }
        if (c0 == 0) {
            D1 = (double)s1;
            D2 = (double)s2;
            D3 = (double)s3;
            D4 = (double)s4;
            DE = (double)ent;
        } else {
            D1 += (double)s1;
            D2 += (double)s2;
            D3 += (double)s3;
            D4 += (double)s4;
            DE += (double)ent;
        }
    }
    const R sc = x0 ? R(1) : R(4);
    const R lo2 = (R(1) - eps) * (R(1) - eps) / sc, hi2 = (R(1) + eps) * (R(1) + eps) / sc;
    unsigned cnt = 0u;
    R gap = mx;
    if (mx > lo2) {
        gap = R(-1);
        auto test = [&](R t) {
            cnt += (t > lo2 && t < hi2) ? 1u : 0u;
            gap = fmax(gap, t <= lo2 ? t : R(-1));
        };
        if (x0) {
#pragma unroll
            for (int j = 0; j < (1 << RL); ++j) {
                const R u = re[j] + im[j], v = re[j] - im[j];
                test(u * u);
                test(v * v);
            }
        } else {
#pragma unroll
            for (int j = 0; j < (1 << RL); ++j) {
                test(re[j] * re[j]);
                test(im[j] * im[j]);
            }
        }
    }
    AccD d;
    const double scd = (double)sc;
    d.s1 = scd * D1;
    d.s2 = scd * scd * D2;
    d.s3 = scd * scd * scd * D3;
    d.s4 = scd * scd * scd * scd * D4;
    d.ent = x0 ? DE : 4.0 * DE + 8.0 * D1;
    d.gap = gap >= R(0) ? scd * (double)gap : -1.0;
    d.cnt = cnt;
    return d;
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

// Fixed-order workgroup reduction; the total is valid in thread 0.  Each wave
// first reduces by shuffles over the values in use (moments up to MOM).
template <int NT, int MOM>
__device__ AccD block_reduce(AccD a, AccD* sh) {
    constexpr int WS = NT < 64 ? NT : 64;
#pragma unroll
    for (int off = WS / 2; off > 0; off >>= 1) {
        a.s1 += __shfl_xor(a.s1, off);
        a.ent += __shfl_xor(a.ent, off);
        a.s2 += __shfl_xor(a.s2, off);
        if constexpr (MOM >= 3) a.s3 += __shfl_xor(a.s3, off);
        if constexpr (MOM >= 4) a.s4 += __shfl_xor(a.s4, off);
        a.gap = fmax(a.gap, __shfl_xor(a.gap, off));
        a.cnt += __shfl_xor(a.cnt, off);
    }
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

// Raw per-workgroup sums, stored in the FamilyRes layout (gap as |F|^2).
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

// ---------------------------------------------------------------------------
// Kernels
// ---------------------------------------------------------------------------

// Whole family in one workgroup (n - 1 = K).  Grid: one block per family.
template <typename R, int TL, int RL, int MOM>
__global__ void __launch_bounds__(1 << TL)
k_fused(const cx<R>* __restrict__ psi, const uint64_t* __restrict__ fpsi, int n, const uint64_t* __restrict__ xs,
        uint64_t x0, R eps, FamilyRes* __restrict__ out) {
    constexpr int K = TL + RL;
    constexpr int NT = 1 << TL;
    __shared__ cx<R> lds[Lds<K>::elems];
    __shared__ AccD shw[NT / 64 > 0 ? NT / 64 : 1];
    __shared__ Lg2Entry lg2t[Lg2Shared<R>::n];
    const uint32_t slot = blockIdx.x;
    const uint64_t x = (xs ? xs[slot] : x0 + slot) & ((1ull << n) - 1ull);  // device lists: x mod 2^n
    R re[1 << RL], im[1 << RL];
    load_products<R, TL, RL>(state_of(psi, fpsi, slot), n - 1, (uint32_t)x, 0u, re, im);
    if constexpr (sizeof(R) == 8) lg2_table_init(lg2t);
    tile_fwht<R, TL, RL, 0>(re, im, lds);
    const AccD tot = block_reduce<NT, MOM>(reduce_points<R, RL, MOM>(re, im, x == 0, eps, lg2t), shw);
    if (threadIdx.x == 0) out[slot] = finish<MOM>(tot, x, n);
}

// Family of x_A for the reduced state (one workgroup per family, n_a - 1 = K).
template <typename R, int TL, int RL, int MOM>
__global__ void __launch_bounds__(1 << TL)
k_fused_reduced(const cx<R>* __restrict__ rho, int na, uint64_t x0, R eps, FamilyRes* __restrict__ out) {
    constexpr int K = TL + RL;
    constexpr int NT = 1 << TL;
    __shared__ cx<R> lds[Lds<K>::elems];
    __shared__ AccD shw[NT / 64 > 0 ? NT / 64 : 1];
    __shared__ Lg2Entry lg2t[Lg2Shared<R>::n];
    const uint32_t slot = blockIdx.x;
    const uint64_t x = x0 + slot;
    R re[1 << RL], im[1 << RL];
    load_reduced<R, TL, RL>(rho, na, (uint32_t)x, 0u, re, im);
    if constexpr (sizeof(R) == 8) lg2_table_init(lg2t);
    tile_fwht<R, TL, RL, 0>(re, im, lds);
    const AccD tot = block_reduce<NT, MOM>(reduce_points<R, RL, MOM>(re, im, x == 0, eps, lg2t), shw);
    if (threadIdx.x == 0) out[slot] = finish<MOM>(tot, x, na);
}

// One 16 x 16 x 4 matrix-core step (accumulator += A B) in the transform precision.  Operands: lane l
// gives A[l mod 16][l / 16] and B[l / 16][l mod 16]; result element v of lane l is
// D[i][l mod 16] with i = 4 (l / 16) + v (FP32) or l / 16 + 4 v (FP64).
typedef float mf4 __attribute__((ext_vector_type(4)));
typedef double md4 __attribute__((ext_vector_type(4)));
template <typename R> struct Mfma;
template <> struct Mfma<float> {
    typedef mf4 acc;
    static __device__ __forceinline__ acc step(float a, float b, acc c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lane, int v) { return 4 * (lane >> 4) + v; }
};
template <> struct Mfma<double> {
    typedef md4 acc;
    static __device__ __forceinline__ acc step(double a, double b, acc c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lane, int v) { return (lane >> 4) + 4 * v; }
};

// rho_A[a, a'] = sum_e psi(a + e d_A) conj(psi(a' + e d_A)) on the matrix cores, written to
// the family-major D (above): one workgroup per 64 x 64 tile of rho_A on and above the
// diagonal (blocks below it return at once; rho_A is Hermitian), wave w the 32 x 32
// quarter (rows 32 (w / 2), columns 32 (w mod 2)) as 2 x 2 blocks of 16 x 16.  Per 4
// values of e a block takes the four real products of
//   re += Ar Br^T + Ai Bi^T,  im += Ai Br^T - Ar Bi^T
// (FP64), or three (FP32, below).
// e runs in chunks of 16 through two LDS buffers: the next chunk's loads are issued into
// registers before the current chunk's products and stored to the other buffer after
// them, so one barrier per chunk separates both uses of a buffer.
template <typename R>
__global__ void __launch_bounds__(256)
k_rho(const cx<R>* __restrict__ psi, int na, int ne, cx<R>* __restrict__ D) {
    constexpr int LD = 64 + 4;   // row pitch of a staged chunk (4 elements of padding)
    constexpr int CH = 16 * LD;  // one staged chunk of 16 values of e
    constexpr int OP = 64 + 1;   // row pitch of the output block staged at the end
    static_assert(64 * OP <= 4 * CH, "the output block reuses the chunk buffers");
    __shared__ cx<R> sh[4 * CH];
    auto ta = [&](int buf, int e, int a) -> cx<R>& { return sh[buf * CH + e * LD + a]; };
    auto tb = [&](int buf, int e, int a) -> cx<R>& { return sh[(2 + buf) * CH + e * LD + a]; };
    if (blockIdx.y > blockIdx.x) return;
    const uint32_t dA = 1u << na;
    const uint64_t dE = 1ull << ne;
    const uint32_t r0 = blockIdx.y * 64, c0 = blockIdx.x * 64;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int wr = 32 * (w >> 1), wc = 32 * (w & 1);
    // thread t stages elements l = t + 256 k (k < 4) of each 16 x 64 chunk: e = l >> 6, a = l & 63
    const int aa = threadIdx.x & 63, ee0 = threadIdx.x >> 6;
    cx<R> pa[4], pb[4];
    auto fetch = [&](uint64_t e0) {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const uint64_t e = e0 + (uint64_t)(ee0 + 4 * k);
            pa[k].re = pa[k].im = pb[k].re = pb[k].im = R(0);
            if (e < dE) {
                if (r0 + aa < dA) pa[k] = psi[(size_t)(r0 + aa) + (e << na)];
                if (c0 + aa < dA) pb[k] = psi[(size_t)(c0 + aa) + (e << na)];
            }
        }
    };
    auto stage = [&](int buf) {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            ta(buf, ee0 + 4 * k, aa) = pa[k];
            tb(buf, ee0 + 4 * k, aa) = pb[k];
        }
    };
    // FP32: three real products per block (Gauss): t1 = Ar Br^T, t2 = Ai Bi^T,
    // t3 = (Ar + Ai)(Br - Bi)^T; then re = t1 + t2, im = t3 - t1 + t2.  FP64 keeps the
    // four products (t1 = re, t2 = im): a third accumulator set would leave one wave per
    // SIMD.
    constexpr bool GAUSS = sizeof(R) == 4;
    typename Mfma<R>::acc t1[2][2], t2[2][2], t3[GAUSS ? 2 : 1][2];
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                t1[bi][bj][v] = t2[bi][bj][v] = R(0);
                if constexpr (GAUSS) t3[bi][bj][v] = R(0);
            }
    fetch(0);
    stage(0);
    __syncthreads();
    int buf = 0;
    const int kl = lane >> 4, il = lane & 15;
    for (uint64_t e0 = 0; e0 < dE; e0 += 16) {
        const bool more = e0 + 16 < dE;
        if (more) fetch(e0 + 16);
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) {
            const int e = 4 * ks + kl;
            R ar[2], ai[2], br[2], bim[2];
#pragma unroll
            for (int b = 0; b < 2; ++b) {
                const cx<R> va = ta(buf, e, wr + 16 * b + il);
                const cx<R> vb = tb(buf, e, wc + 16 * b + il);
                ar[b] = va.re;
                ai[b] = va.im;
                br[b] = vb.re;
                bim[b] = vb.im;
            }
            // the products in turn over the accumulators, so that consecutive steps never
            // wait on each other's results
            if constexpr (GAUSS) {
#pragma unroll
                for (int bi = 0; bi < 2; ++bi)
#pragma unroll
                    for (int bj = 0; bj < 2; ++bj) t1[bi][bj] = Mfma<R>::step(ar[bi], br[bj], t1[bi][bj]);
#pragma unroll
                for (int bi = 0; bi < 2; ++bi)
#pragma unroll
                    for (int bj = 0; bj < 2; ++bj) t2[bi][bj] = Mfma<R>::step(ai[bi], bim[bj], t2[bi][bj]);
#pragma unroll
                for (int bi = 0; bi < 2; ++bi)
#pragma unroll
                    for (int bj = 0; bj < 2; ++bj)
                        t3[bi][bj] = Mfma<R>::step(ar[bi] + ai[bi], br[bj] - bim[bj], t3[bi][bj]);
            } else {
#pragma unroll
                for (int p = 0; p < 2; ++p)
#pragma unroll
                    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
                        for (int bj = 0; bj < 2; ++bj) {
                            t1[bi][bj] = Mfma<R>::step(p ? ai[bi] : ar[bi], p ? bim[bj] : br[bj], t1[bi][bj]);
                            t2[bi][bj] = Mfma<R>::step(p ? -ar[bi] : ai[bi], p ? bim[bj] : br[bj], t2[bi][bj]);
                        }
            }
        }
        if (more) {
            // the other buffer was last read in the previous chunk, before the barrier
            // that closed it
            stage(buf ^ 1);
            __syncthreads();
            buf ^= 1;
        }
    }
    // The tile T = rho_A[r0 + ri, c0 + ci] goes to D through LDS: entry (ri, ci) belongs to
    // family x = r ^ c at a = c, and its mirror conj T (rho_A is Hermitian) to the same
    // family at a = r.  With R = r0 / 64, C = c0 / 64 the first fills the 64 x 64 block
    // (R ^ C, C) of D at (ri ^ ci, ci), the second (off the diagonal) the block (R ^ C, R) at
    // (ri ^ ci, ri); every block of D is written by exactly one workgroup, row by row.
    __syncthreads();   // every wave is done with the chunk buffers
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                cx<R> o;
                if constexpr (GAUSS) {
                    o.re = t1[bi][bj][v] + t2[bi][bj][v];
                    o.im = (t3[bi][bj][v] - t1[bi][bj][v]) + t2[bi][bj][v];
                } else {
                    o.re = t1[bi][bj][v];
                    o.im = t2[bi][bj][v];
                }
                sh[(wr + 16 * bi + Mfma<R>::row(lane, v)) * OP + wc + 16 * bj + il] = o;
            }
    __syncthreads();
    const uint32_t xb = (blockIdx.y ^ blockIdx.x) * 64;
    for (int idx = threadIdx.x; idx < 64 * 64; idx += 256) {
        const uint32_t xl = (uint32_t)idx >> 6, cl = (uint32_t)idx & 63u;
        const uint32_t x = xb + xl, a = c0 + cl;
        if (x < dA && a < dA) D[(size_t)x * dA + a] = sh[(xl ^ cl) * OP + cl];
    }
    if (blockIdx.y != blockIdx.x) {
        for (int idx = threadIdx.x; idx < 64 * 64; idx += 256) {
            const uint32_t xl = (uint32_t)idx >> 6, rl = (uint32_t)idx & 63u;
            const uint32_t x = xb + xl, a = r0 + rl;
            if (x < dA && a < dA) {
                cx<R> v = sh[rl * OP + (xl ^ rl)];
                v.im = -v.im;
                D[(size_t)x * dA + a] = v;
            }
        }
    }
}

// Intermediate tiles of the 2^15-point plans belong to families of 2^21 and more
// points, far beyond what the caches hold between passes: those passes move them
// with streaming (nontemporal) loads and stores.  Smaller plans keep the default
// policy, under which part of a batch is still cached when the next pass reads it.
template <bool STREAM, typename R>
__device__ __forceinline__ void st_point(cx<R>* p, R re, R im) {
    if constexpr (STREAM) {
        __builtin_nontemporal_store(re, &p->re);
        __builtin_nontemporal_store(im, &p->im);
    } else {
        cx<R> v;
        v.re = re;
        v.im = im;
        *p = v;
    }
}

template <bool STREAM, typename R>
__device__ __forceinline__ void ld_point(const cx<R>* p, R& re, R& im) {
    if constexpr (STREAM) {
        re = __builtin_nontemporal_load(&p->re);
        im = __builtin_nontemporal_load(&p->im);
    } else {
        const cx<R> v = *p;
        re = v.re;
        im = v.im;
    }
}

template <typename R, int TL, int RL, bool STREAM = false>
__device__ __forceinline__ void store_tile(cx<R>* __restrict__ dst, const R (&re)[1 << RL], const R (&im)[1 << RL]) {
    constexpr int A = final_window<TL, RL, 0>();
    cx<R>* p = dst + thread_part<A, RL>(threadIdx.x);
#pragma unroll
    for (int j = 0; j < (1 << RL); ++j) st_point<STREAM>(p + ((uint32_t)j << A), re[j], im[j]);
}

// Half spectrum G of one family written out (signed values of small states).
template <typename R, int TL, int RL>
__global__ void __launch_bounds__(1 << TL)
k_fused_store(const cx<R>* __restrict__ psi, int n, uint64_t x, cx<R>* __restrict__ G) {
    constexpr int K = TL + RL;
    __shared__ cx<R> lds[Lds<K>::elems];
    R re[1 << RL], im[1 << RL];
    load_products<R, TL, RL>(psi, n - 1, (uint32_t)x, 0u, re, im);
    tile_fwht<R, TL, RL, 0>(re, im, lds);
    store_tile<R, TL, RL>(G, re, im);
}

// First pass of a multi-pass transform: products + low K index bits of one tile.
// HSRC: the values come from the family-major reduced density matrix of the mixed-state
// path (psi is D and n is n_a) instead of products of the state.
// Grid: (tiles per family, families), or with GRP > 1 (states of 16 MiB and more, families
// in groups of GRP with the same top bit of x, hence the same state tiles): one dimension
// of tiles x ceil(nb / GRP) GRP workgroups, numbered so that the GRP workgroups of one
// tile and group follow each other on one XCD (workgroups are dealt round-robin to the 8
// XCDs): the first reads the tile from HBM or the MALL, the others find it in that XCD's L2.
// Requires tiles % 8 == 0; workgroups of the padding slots (>= nb) return at once.
template <typename R, int TL, int RL, bool SPLIT = false, bool HSRC = false, int GRP = 1>
__global__ void __launch_bounds__(1 << TL)
k_first(const cx<R>* __restrict__ psi, const uint64_t* __restrict__ fpsi, int n, const uint64_t* __restrict__ xs,
        uint64_t x0, cx<R>* __restrict__ work, int nb) {
    constexpr int K = TL + RL;
    __shared__ __align__(16) char lds[LdsBytes<R, K, SPLIT, RL>::v];
    const int nh = n - 1;
    uint32_t tile, slot;
    if constexpr (GRP > 1) {
        const uint32_t t8 = 1u << (nh - K - 3);   // tiles / 8
        const uint32_t s = blockIdx.x >> 3, r = s / GRP;
        tile = ((r & (t8 - 1u)) << 3) | (blockIdx.x & 7u);
        slot = (r >> (nh - K - 3)) * GRP + s % GRP;
        if (slot >= (uint32_t)nb) return;
    } else {
        tile = blockIdx.x;
        slot = blockIdx.y;
    }
    const uint32_t x = (uint32_t)((xs ? xs[slot] : x0 + slot) & ((1ull << n) - 1ull));
    R re[1 << RL], im[1 << RL];
    const cx<R>* ps = state_of(psi, fpsi, slot);
    if constexpr (HSRC) load_reduced<R, TL, RL>(ps, n, x, tile, re, im);
    else if (x >= (1u << K)) load_products_hi<R, TL, RL>(ps, x, tile, re, im);
    else load_products<R, TL, RL>(ps, nh, x, tile, re, im);
    tile_fwht<R, TL, RL, 0, SPLIT>(re, im, lds);
    store_tile<R, TL, RL, SPLIT>(work + ((size_t)slot << nh) + ((size_t)tile << K), re, im);
}

// v from lane (lane XOR 2^B) of the same wave, B < 4, by DPP row permutations
// (plain VALU moves, no LDS): xor 1 and xor 2 are quad permutations, xor 8 is a
// rotation of the 16-lane row by 8, xor 4 is the 8-lane mirror (xor 7) followed
// by the quad reversal (xor 3).
template <int B>
__device__ __forceinline__ uint32_t dpp_xor(uint32_t w) {
    const int v = (int)w;
    if constexpr (B == 0) return (uint32_t)__builtin_amdgcn_mov_dpp(v, 0xB1, 0xF, 0xF, true);
    if constexpr (B == 1) return (uint32_t)__builtin_amdgcn_mov_dpp(v, 0x4E, 0xF, 0xF, true);
    if constexpr (B == 2) return (uint32_t)__builtin_amdgcn_mov_dpp(__builtin_amdgcn_mov_dpp(v, 0x141, 0xF, 0xF, true),
                                                                    0x1B, 0xF, 0xF, true);
    if constexpr (B == 3) return (uint32_t)__builtin_amdgcn_mov_dpp(v, 0x128, 0xF, 0xF, true);
    return w;
}

template <int B, typename R>
__device__ __forceinline__ R lane_xor(R v) {
    constexpr int NW = sizeof(R) / 4;
    uint32_t w[NW];
    __builtin_memcpy(w, &v, sizeof(R));
#pragma unroll
    for (int k = 0; k < NW; ++k) w[k] = dpp_xor<B>(w[k]);
    __builtin_memcpy(&v, w, sizeof(R));
    return v;
}

template <int B, typename R, int RL>
__device__ __forceinline__ void regs_lane_xor(R (&vr)[1 << RL], R (&vi)[1 << RL]) {
#pragma unroll
    for (int j = 0; j < (1 << RL); ++j) {
        vr[j] = lane_xor<B>(vr[j]);
        vi[j] = lane_xor<B>(vi[j]);
    }
}

// First pass for a run of fam <= 16 consecutive families x = x_r + f (x_r a
// multiple of fam, f < fam) that share x >> K != 0 (exact sweeps).  The state
// tile tu << K and its partner (tu ^ (x >> K)) << K are the same for the whole
// run and both stay in registers: thread t holds psi at t of its own tile and at
// (t ^ (x_r mod 2^TL)) + ((j ^ jx) << TL) of the partner tile, jx = (x_r mod 2^K) >> TL.
// Family f needs the partner value of lane t ^ f, in the same 16-lane row; the
// families are taken in Gray-code order so that each step moves the partner
// registers by one lane XOR.  Grid: (tiles, run / fam).
template <typename R, int TL, int RL>
__global__ void __launch_bounds__(1 << TL)
k_first_shared(const cx<R>* __restrict__ psi, int n, uint64_t x0, int fam, cx<R>* __restrict__ work) {
    constexpr int K = TL + RL;
    static_assert(TL >= 6, "a 16-lane row must lie inside one wave");
    __shared__ cx<R> lds[Lds<K>::elems];
    const int nh = n - 1;
    const uint32_t tile = blockIdx.x, grp = blockIdx.y;
    const uint32_t slot0 = grp * (uint32_t)fam;
    const uint32_t xr = (uint32_t)(x0 + slot0);
    const uint32_t xh = xr >> K;
    const int q = 31 - __builtin_clz(xh);
    const uint32_t lowm = (1u << q) - 1u;
    const uint32_t tu = (tile & lowm) | ((tile & ~lowm) << 1);
    const uint32_t tv = tu ^ xh;
    const uint32_t c = xr & ((1u << TL) - 1u);
    const uint32_t jx = (xr & ((1u << K) - 1u)) >> TL;
    const uint32_t tid = threadIdx.x;
    R ur[1 << RL], ui[1 << RL], vr[1 << RL], vi[1 << RL];
    {
        const cx<R>* pa = psi + ((size_t)tu << K) + tid;
        const cx<R>* pv = psi + ((size_t)tv << K) + (tid ^ c);
#pragma unroll
        for (int j = 0; j < (1 << RL); ++j) {
            const cx<R> u = pa[(uint32_t)j << TL];
            const cx<R> v = pv[((uint32_t)j ^ jx) << TL];
            ur[j] = u.re;
            ui[j] = u.im;
            vr[j] = v.re;
            vi[j] = v.im;
        }
    }
    for (int k = 0; k < fam; ++k) {
        const uint32_t slot = slot0 + ((uint32_t)k ^ ((uint32_t)k >> 1));
        R re[1 << RL], im[1 << RL];
#pragma unroll
        for (int j = 0; j < (1 << RL); ++j) {
            re[j] = ur[j] * vr[j] + ui[j] * vi[j];
            im[j] = ur[j] * vi[j] - ui[j] * vr[j];
        }
        tile_fwht<R, TL, RL, 0, false, true>(re, im, lds);
        store_tile<R, TL, RL>(work + ((size_t)slot << nh) + ((size_t)tile << K), re, im);
        if (k + 1 < fam) {
            switch (__builtin_ctz((unsigned)(k + 1))) {
                case 0: regs_lane_xor<0, R, RL>(vr, vi); break;
                case 1: regs_lane_xor<1, R, RL>(vr, vi); break;
                case 2: regs_lane_xor<2, R, RL>(vr, vi); break;
                default: regs_lane_xor<3, R, RL>(vr, vi); break;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Split-BF16 Hadamard blocks on the matrix cores
// ---------------------------------------------------------------------------
// v_mfma_f32_16x16x32_bf16 (one wave): lane l holds A[l mod 16][8 (l/16) + t] and
// B[8 (l/16) + t][l mod 16], t = 0..7, and gets C[4 (l/16) + v][l mod 16], v = 0..3 (layout
// checked on the device).  A 16 x 16 real block X is kept in the C layout: lane (g, c) =
// (l/16, l mod 16) holds X[4g + v][c] in slot v.  Fed back as A with the K index
// interleaved as k = 2 k16 + s, slot pairs (hi, lo) = the two BF16 parts of X[4g + v][c]
// (x = hi + lo + r, |r| <= 2^-18 |x|), A[i][k16] = X[k16][i], and with B[2 k16 + s][j] =
// H16[k16][j] (exact in BF16) the product is C = X^T H16 in FP32: C[i][j] = (H16 X)[j][i].
// So one step transforms the 4 index bits held in (g, v) and leaves the result with those
// bits in the lane (c) position and the other 4 bits in (g, v); a second step transforms
// those, and the block is back in its starting layout with all 8 bits transformed.
// Within a tile, point i of register (b, v) of lane (g, c) of wave w has index bits
// c + 16 (4 g + v) + 256 (b + B w) before the exchange below.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// H16 as the B operand with the interleaved K index: B[8 g + t][j] = H16[4 g + t / 2][j].
__device__ __forceinline__ bf16x8 h16_operand() {
    const int l = threadIdx.x & 63;
    const int j = l & 15, g = l >> 4;
    bf16x8 h;
#pragma unroll
    for (int t = 0; t < 8; ++t) {
        const int k16 = 4 * g + (t >> 1);
        h[t] = (__popc((unsigned)(k16 & j)) & 1) ? (__bf16)(-1.0f) : (__bf16)1.0f;
    }
    return h;
}

// One H16 step on the 16 x 16 real block x (C layout), hi / lo split, FP32 accumulation.
__device__ __forceinline__ void h16_step(float (&x)[4], const bf16x8& h) {
    bf16x8 a;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const __bf16 hi = (__bf16)x[v];
        const __bf16 lo = (__bf16)(x[v] - (float)hi);
        a[2 * v] = hi;
        a[2 * v + 1] = lo;
    }
    mf4 acc = {0.f, 0.f, 0.f, 0.f};
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, h, acc, 0, 0, 0);
#pragma unroll
    for (int v = 0; v < 4; ++v) x[v] = acc[v];
}

// Tile of 2^(8 + LB + LW) points: W = 2^LW waves, B = 2^LB blocks of 256 points per wave
// (re / im [4 b + v]).  Bits 0..7 by two matrix-core steps per block and component, the
// block bits by FP32 butterflies, then one LDS exchange moves the wave bits into the low
// block-bit positions (LB >= LW) and FP32 butterflies finish them.  After the call, register
// (b, v) of lane (g, c) of wave w holds index
//     c + 16 (4 g + v) + 256 ((b & ~(W - 1)) | w) + 256 B (b & (W - 1)).
template <int LB, int LW>
struct MfmaTile {
    static constexpr int B = 1 << LB, W = 1 << LW, K = 8 + LB + LW;
    static_assert(LB >= LW, "the wave bits are exchanged into block-bit positions");
    static constexpr int N = 4 * B;   // complex values per lane
    // padded LDS index: 16 complex of padding per 64 points, so that the four 16-lane groups
    // of a half wave (128 B each) fall on distinct banks
    static __device__ __forceinline__ uint32_t pad(uint32_t i) { return i + ((i >> 6) << 4); }
    static constexpr int lds_elems = (1 << K) + ((1 << K) >> 2);
    static __device__ __forceinline__ uint32_t index_before(uint32_t w, uint32_t g, uint32_t c, int b, int v) {
        return c + 16u * (4u * g + (uint32_t)v) + 256u * ((uint32_t)b + (uint32_t)B * w);
    }
    static __device__ __forceinline__ uint32_t index_after(uint32_t w, uint32_t g, uint32_t c, int b, int v) {
        const uint32_t bb = ((uint32_t)b & ~(uint32_t)(W - 1)) | w;
        return c + 16u * (4u * g + (uint32_t)v) + 256u * bb + 256u * (uint32_t)B * ((uint32_t)b & (uint32_t)(W - 1));
    }
    static __device__ __forceinline__ void butterflies(float (&re)[N], float (&im)[N], int bit) {
#pragma unroll
        for (int b = 0; b < B; ++b) {
            if (b & bit) continue;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int j = 4 * b + v, k = 4 * (b | bit) + v;
                const float ar = re[j], ai = im[j], br = re[k], bi = im[k];
                re[j] = ar + br;
                im[j] = ai + bi;
                re[k] = ar - br;
                im[k] = ai - bi;
            }
        }
    }
    static __device__ __forceinline__ void run(float (&re)[N], float (&im)[N], cx<float>* lds) {
        const bf16x8 h = h16_operand();
#pragma unroll
        for (int b = 0; b < B; ++b) {
            float tr[4], ti[4];
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                tr[v] = re[4 * b + v];
                ti[v] = im[4 * b + v];
            }
            h16_step(tr, h);
            h16_step(ti, h);
            h16_step(tr, h);
            h16_step(ti, h);
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                re[4 * b + v] = tr[v];
                im[4 * b + v] = ti[v];
            }
        }
#pragma unroll
        for (int bit = 1; bit < B; bit <<= 1) butterflies(re, im, bit);
        if constexpr (LW > 0) {
            const uint32_t l = threadIdx.x & 63, w = threadIdx.x >> 6, g = l >> 4, c = l & 15;
#pragma unroll
            for (int b = 0; b < B; ++b)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    cx<float> t;
                    t.re = re[4 * b + v];
                    t.im = im[4 * b + v];
                    lds[pad(index_before(w, g, c, b, v))] = t;
                }
            __syncthreads();
#pragma unroll
            for (int b = 0; b < B; ++b)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const cx<float> t = lds[pad(index_after(w, g, c, b, v))];
                    re[4 * b + v] = t.re;
                    im[4 * b + v] = t.im;
                }
#pragma unroll
            for (int bit = 1; bit < W; bit <<= 1) butterflies(re, im, bit);
        }
    }
};

// Products of the half-size problem at the tile-local indices of the matrix-core layout
// (before the exchange): half index (tile << K) + index_before(...).
template <class T>
__device__ __forceinline__ void load_products_mfma(const cx<float>* __restrict__ psi, int nh, uint32_t x, uint32_t tile,
                                                   float (&re)[T::N], float (&im)[T::N]) {
    const uint32_t l = threadIdx.x & 63, w = threadIdx.x >> 6, g = l >> 4, c = l & 15;
    if (x != 0u) {
        const int p = 31 - __builtin_clz(x);
        const uint32_t lowmask = (1u << p) - 1u;
#pragma unroll
        for (int b = 0; b < T::B; ++b)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const uint32_t bp = (tile << T::K) + T::index_before(w, g, c, b, v);
                const uint32_t bb = (bp & lowmask) | ((bp & ~lowmask) << 1);
                const cx<float> a = psi[bb];
                const cx<float> q = psi[bb ^ x];
                re[4 * b + v] = a.re * q.re + a.im * q.im;
                im[4 * b + v] = a.re * q.im - a.im * q.re;
            }
    } else {
        const uint32_t half = 1u << nh;
#pragma unroll
        for (int b = 0; b < T::B; ++b)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const uint32_t bp = (tile << T::K) + T::index_before(w, g, c, b, v);
                const cx<float> a = psi[bp];
                const cx<float> q = psi[bp + half];
                re[4 * b + v] = a.re * a.re + a.im * a.im;
                im[4 * b + v] = q.re * q.re + q.im * q.im;
            }
    }
}

// Whole family in one workgroup on the matrix cores (n - 1 = K = 8 + LB + LW).
template <int LB, int LW, int MOM>
__global__ void __launch_bounds__(64 << LW)
k_fused_mfma(const cx<float>* __restrict__ psi, const uint64_t* __restrict__ fpsi, int n,
             const uint64_t* __restrict__ xs, uint64_t x0, float eps, FamilyRes* __restrict__ out) {
    using T = MfmaTile<LB, LW>;
    constexpr int NT = 64 << LW;
    __shared__ cx<float> lds[LW > 0 ? T::lds_elems : 1];
    __shared__ AccD shw[NT / 64];
    const uint32_t slot = blockIdx.x;
    const uint64_t x = (xs ? xs[slot] : x0 + slot) & ((1ull << n) - 1ull);
    float re[T::N], im[T::N];
    load_products_mfma<T>(state_of(psi, fpsi, slot), n - 1, (uint32_t)x, 0u, re, im);
    T::run(re, im, lds);
    constexpr int RL = LB + 2;
    const AccD tot = block_reduce<NT, MOM>(reduce_points<float, RL, MOM>(re, im, x == 0, eps, nullptr), shw);
    if (threadIdx.x == 0) out[slot] = finish<MOM>(tot, x, n);
}

// First pass of a multi-pass transform on the matrix cores: products + the low 12 index
// bits of one tile (4 waves x 4 blocks); the tile is written back in index order.
__global__ void __launch_bounds__(256)
k_first_mfma(const cx<float>* __restrict__ psi, const uint64_t* __restrict__ fpsi, int n,
             const uint64_t* __restrict__ xs, uint64_t x0, cx<float>* __restrict__ work) {
    using T = MfmaTile<2, 2>;
    __shared__ cx<float> lds[T::lds_elems];
    const int nh = n - 1;
    const uint32_t tile = blockIdx.x, slot = blockIdx.y;
    const uint32_t x = (uint32_t)((xs ? xs[slot] : x0 + slot) & ((1ull << n) - 1ull));
    float re[T::N], im[T::N];
    load_products_mfma<T>(state_of(psi, fpsi, slot), nh, x, tile, re, im);
    T::run(re, im, lds);
    const uint32_t l = threadIdx.x & 63, w = threadIdx.x >> 6, g = l >> 4, c = l & 15;
    cx<float>* dst = work + ((size_t)slot << nh) + ((size_t)tile << T::K);
#pragma unroll
    for (int b = 0; b < T::B; ++b)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            cx<float> t;
            t.re = re[4 * b + v];
            t.im = im[4 * b + v];
            dst[T::index_after(w, g, c, b, v)] = t;
        }
}

// Column pass over index bits [lo, lo + S) of every family in the batch.
// A tile is 2^S rows (stride 2^lo) by 2^W consecutive columns, W = K - S.
// Grid: (2^(nh - K), families).  LAST: reduce to one partial per workgroup
// (parts[family][block]) instead of writing the spectrum back.
// SPLIT: the exchange moves real then imaginary parts through one buffer of half the
// size; STREAM: nontemporal loads and stores (tiles far beyond what the caches hold).
// PF > 0 (single-precision reducing passes of one workgroup per CU): each workgroup takes
// two tiles, bid and bid + gridDim.x, and issues the loads of the second tile's first PF
// points (per thread) before it reduces the first, so that those loads overlap the
// reductions, which nothing else on the CU would.  Each tile's arithmetic is unchanged.
template <typename R, int TL, int RL, int S, bool LAST, int MOM, bool SPLIT = false, bool STREAM = SPLIT, int PF = 0>
__global__ void __launch_bounds__(1 << TL)
k_column(cx<R>* __restrict__ work, int n, int lo, const uint64_t* __restrict__ xs, uint64_t x0, R eps,
         FamilyRes* __restrict__ parts) {
    constexpr int K = TL + RL;
    constexpr int NT = 1 << TL;
    constexpr int W = K - S;
    __shared__ __align__(16) char lds[LdsBytes<R, K, SPLIT, RL>::v];
    const int nh = n - 1;
    const int cbits = lo - W;
    if constexpr (PF > 0) {
        // block_reduce's barrier (NT > 64) separates the first tile's last LDS reads from the
        // second tile's first LDS writes
        static_assert(LAST && sizeof(R) == 4 && NT > 64 && PF <= (1 << RL), "two-tile reducing pass");
        const uint32_t GX = gridDim.x;
        const uint32_t bid = (GX & 7u) ? blockIdx.x : (blockIdx.x & 7u) * (GX >> 3) + (blockIdx.x >> 3);
        const uint32_t slot = blockIdx.y;
        const uint32_t tid = threadIdx.x;
        constexpr uint32_t WM = (1u << W) - 1u;
        auto tile_at = [&](uint32_t t) -> const cx<R>* {
            const uint32_t cb = t & ((1u << cbits) - 1u), hb = t >> cbits;
            return work + ((size_t)slot << nh) + ((size_t)hb << (lo + S)) + ((size_t)cb << W) + (tid & WM) +
                   ((size_t)(tid >> W) << lo);
        };
        // point offsets from a row shift the compiler cannot see through, taken anew for each
        // group of loads (otherwise it keeps 64 scalar offsets live across both tiles)
        auto at = [&](int j, int sh) -> size_t {
            const uint32_t J = (uint32_t)j << TL;
            return (J & WM) + ((size_t)(J >> W) << sh);
        };
        auto fresh = [&]() {
            int v = lo;
            asm volatile("" : "+s"(v));
            return v;
        };
        const uint64_t x = (xs ? xs[slot] : x0 + slot) & ((1ull << n) - 1ull);
        __shared__ AccD shw[NT / 64];
        R re[1 << RL], im[1 << RL], pre[PF], pim[PF];
        const cx<R>* p0 = tile_at(bid);
        const cx<R>* p1 = tile_at(bid + GX);
        const int l0 = fresh();
#pragma unroll
        for (int j = 0; j < (1 << RL); ++j) ld_point<STREAM>(p0 + at(j, l0), re[j], im[j]);
        tile_fwht<R, TL, RL, W, SPLIT, false, true>(re, im, lds);
        const int l1 = fresh();
#pragma unroll
        for (int j = 0; j < PF; ++j) ld_point<STREAM>(p1 + at(j, l1), pre[j], pim[j]);
        asm volatile("" ::: "memory");   // those loads stay above the reductions
        AccD tot = block_reduce<NT, MOM>(reduce_points<R, RL, MOM>(re, im, x == 0, eps, nullptr), shw);
        if (tid == 0) parts[(size_t)slot * (2u * GX) + bid] = raw_res(tot, x);
#pragma unroll
        for (int j = 0; j < PF; ++j) {
            re[j] = pre[j];
            im[j] = pim[j];
        }
        const int l2 = fresh();
#pragma unroll
        for (int j = PF; j < (1 << RL); ++j) ld_point<STREAM>(p1 + at(j, l2), re[j], im[j]);
        tile_fwht<R, TL, RL, W, SPLIT, false, true>(re, im, lds);
        tot = block_reduce<NT, MOM>(reduce_points<R, RL, MOM>(re, im, x == 0, eps, nullptr), shw);
        if (tid == 0) parts[(size_t)slot * (2u * GX) + bid + GX] = raw_res(tot, x);
        return;
    }
    // Workgroups are dealt round-robin to the 8 XCDs; when a family has a multiple of
    // 8 blocks, renumber them so that each XCD takes a contiguous range of column
    // blocks and neighbouring (partial-cache-line) columns share its L2.
    const uint32_t G = gridDim.x;
    const uint32_t bid = (G & 7u) ? blockIdx.x : (blockIdx.x & 7u) * (G >> 3) + (blockIdx.x >> 3);
    const uint32_t slot = blockIdx.y;
    const uint32_t cb = bid & ((1u << cbits) - 1u);
    const uint32_t hb = bid >> cbits;
    cx<R>* base = work + ((size_t)slot << nh) + ((size_t)hb << (lo + S)) + ((size_t)cb << W);
    const uint32_t tid = threadIdx.x;
    constexpr uint32_t WM = (1u << W) - 1u;
    // Point i = T | J (thread part T, register part J = j 2^A, disjoint bits) sits at
    // column i mod 2^W and row i >> W: a per-thread base plus, for each j, a
    // compile-time column offset and a compile-time number of rows.
    const cx<R>* pin = base + (tid & WM) + ((size_t)(tid >> W) << lo);
    R re[1 << RL], im[1 << RL];
#pragma unroll
    for (int j = 0; j < (1 << RL); ++j) {
        const uint32_t J = (uint32_t)j << TL;
        ld_point<STREAM>(pin + (J & WM) + ((size_t)(J >> W) << lo), re[j], im[j]);
    }
    // the FP64 log2 table of the reductions, filled while the loads are in flight
    __shared__ Lg2Entry lg2t[LAST ? Lg2Shared<R>::n : 1];
    if constexpr (LAST && sizeof(R) == 8) lg2_table_init(lg2t);
    tile_fwht<R, TL, RL, W, SPLIT, false, true>(re, im, lds);
    if constexpr (!LAST) {
        constexpr int A = final_window<TL, RL, W>();
        const uint32_t T = thread_part<A, RL>(tid);
        cx<R>* pout = base + (T & WM) + ((size_t)(T >> W) << lo);
#pragma unroll
        for (int j = 0; j < (1 << RL); ++j) {
            const uint32_t J = (uint32_t)j << A;
            st_point<STREAM>(pout + (J & WM) + ((size_t)(J >> W) << lo), re[j], im[j]);
        }
    } else {
        __shared__ AccD shw[NT / 64 > 0 ? NT / 64 : 1];
        const uint64_t x = (xs ? xs[slot] : x0 + slot) & ((1ull << n) - 1ull);
        const AccD tot = block_reduce<NT, MOM>(reduce_points<R, RL, MOM>(re, im, x == 0, eps, lg2t), shw);
        if (threadIdx.x == 0) parts[(size_t)slot * G + bid] = raw_res(tot, x);
    }
}

// Stable counting sort of a list of at most 4096 families by the top set bit of
// x mod 2^n (x = 0 first): xs_sorted[j] = xs[perm[j]].  One wave; lane t takes a
// contiguous chunk of the list and keeps its key counts in its own column of h.
__global__ void __launch_bounds__(64)
k_sort_top(const uint64_t* __restrict__ xs, int n, int nx, uint64_t* __restrict__ xs_sorted,
           uint32_t* __restrict__ perm) {
    constexpr int NK = 33;   // keys 0 (x = 0) and 1..32 (top bit + 1)
    __shared__ uint32_t h[NK][64];
    const int t = threadIdx.x;
    const int per = (nx + 63) / 64;
    const int i0 = min(nx, t * per), i1 = min(nx, i0 + per);
    const uint64_t mask = (1ull << n) - 1ull;
    for (int k = 0; k < NK; ++k) h[k][t] = 0u;
    for (int i = i0; i < i1; ++i) {
        const uint64_t x = xs[i] & mask;
        ++h[x ? 64 - __clzll((long long)x) : 0][t];
    }
    // exclusive prefix over (key, lane) in key-major order
    uint32_t base = 0;
    for (int k = 0; k < NK; ++k) {
        const uint32_t v = h[k][t];
        uint32_t incl = v;
        for (int d = 1; d < 64; d <<= 1) {
            const uint32_t o = __shfl_up(incl, d);
            if (t >= d) incl += o;
        }
        h[k][t] = base + incl - v;
        base += __shfl(incl, 63);
    }
    for (int i = i0; i < i1; ++i) {
        const uint64_t x = xs[i] & mask;
        const uint32_t j = h[x ? 64 - __clzll((long long)x) : 0][t]++;
        xs_sorted[j] = xs[i];
        perm[j] = (uint32_t)i;
    }
}

__global__ void __launch_bounds__(256)
k_scatter_res(const FamilyRes* __restrict__ in, const uint32_t* __restrict__ perm, int nx, FamilyRes* __restrict__ out) {
    const int j = (int)(blockIdx.x * 256u + threadIdx.x);
    if (j < nx) out[perm[j]] = in[j];
}

// Neumaier's compensated sum: s holds the running total, c the low-order parts that the
// additions lost; the sum is s + c.
__device__ __forceinline__ void comp_add(double& s, double& c, double v) {
    const double t = s + v;
    c += fabs(s) >= fabs(v) ? (s - t) + v : (v - t) + s;
    s = t;
}

// Per-family fixed-order sum of the final pass's partials.  Grid: one workgroup of NT
// threads per family (one wave, or four for families of 16384 partials and more).  Each
// thread's run over the partials is compensated; the tree above it is not.
template <int MOM, int NT>
__global__ void __launch_bounds__(NT)
k_finalize(const FamilyRes* __restrict__ parts, int nblk, int n, FamilyRes* __restrict__ out) {
    const FamilyRes* p = parts + (size_t)blockIdx.x * nblk;
    AccD a;
    a.s1 = a.ent = a.s2 = a.s3 = a.s4 = 0.0;
    a.gap = -1.0;
    a.cnt = 0u;
    double c1 = 0.0, ce = 0.0, c2 = 0.0, c3 = 0.0, c4 = 0.0;
    for (int i = threadIdx.x; i < nblk; i += NT) {
        const AccD b = acc_of(p[i]);
        comp_add(a.s1, c1, b.s1);
        comp_add(a.ent, ce, b.ent);
        comp_add(a.s2, c2, b.s2);
        comp_add(a.s3, c3, b.s3);
        comp_add(a.s4, c4, b.s4);
        a.gap = fmax(a.gap, b.gap);
        a.cnt += b.cnt;
    }
    a.s1 += c1;
    a.ent += ce;
    a.s2 += c2;
    a.s3 += c3;
    a.s4 += c4;
    if constexpr (NT == 64) {
        a = wave_reduce<64>(a);
    } else {
        __shared__ AccD sh[NT / 64];
        a = block_reduce<NT, MOM>(a, sh);
    }
    if (threadIdx.x == 0) out[blockIdx.x] = finish<MOM>(a, p[0].x, n);
}

// Launch of k_finalize for nfam families of nblk partials each.
template <int MOM>
void launch_finalize(const FamilyRes* parts, int nblk, int n, int64_t nfam, FamilyRes* out, hipStream_t st) {
    if (nblk >= 16384)
        hipLaunchKernelGGL((k_finalize<MOM, 256>), dim3((unsigned)nfam), dim3(256), 0, st, parts, nblk, n, out);
    else
        hipLaunchKernelGGL((k_finalize<MOM, 64>), dim3((unsigned)nfam), dim3(64), 0, st, parts, nblk, n, out);
}

__device__ __forceinline__ void zero_sums(SweepSums& t) {
    t.S[0] = t.S[1] = t.S[2] = t.L = t.P = 0.0;
    t.gap = -1.0;
    t.nu_cnt = 0;
    t.count = 0;
    for (int a = 0; a < 3; ++a) t.Snz[a] = t.Q[a] = 0.0;
    t.pad[0] = t.pad[1] = 0.0;
}

__device__ __forceinline__ void add_sums(SweepSums& a, const SweepSums& b) {
    a.S[0] += b.S[0];
    a.S[1] += b.S[1];
    a.S[2] += b.S[2];
    a.L += b.L;
    a.P += b.P;
    a.gap = fmax(a.gap, b.gap);
    a.nu_cnt += b.nu_cnt;
    a.count += b.count;
    for (int k = 0; k < 3; ++k) {
        a.Snz[k] += b.Snz[k];
        a.Q[k] += b.Q[k];
    }
}

// Compensated run of one thread over SweepSums values (the sums of each field).
struct SweepComp {
    double S[3], L, P, Snz[3], Q[3];
};

__device__ __forceinline__ void zero_comp(SweepComp& c) {
    for (int a = 0; a < 3; ++a) c.S[a] = c.Snz[a] = c.Q[a] = 0.0;
    c.L = c.P = 0.0;
}

__device__ __forceinline__ void fold_comp(SweepSums& t, const SweepComp& c) {
    for (int a = 0; a < 3; ++a) {
        t.S[a] += c.S[a];
        t.Snz[a] += c.Snz[a];
        t.Q[a] += c.Q[a];
    }
    t.L += c.L;
    t.P += c.P;
}

// Fixed-order sums of per-family results: block b sums families [b F, (b+1) F) of the
// count, F = FAM_PER_SLOT, into out[b].  Each thread's run is compensated, the block
// tree (8 levels) is not.
__global__ void __launch_bounds__(256)
k_reduce_fam(const FamilyRes* __restrict__ in, int64_t count, SweepSums* __restrict__ out) {
    constexpr int NT = 256;
    __shared__ SweepSums sh[NT];
    SweepSums t;
    zero_sums(t);
    SweepComp c;
    zero_comp(c);
    const int64_t b0 = (int64_t)blockIdx.x * FAM_PER_SLOT;
    const int64_t b1 = b0 + FAM_PER_SLOT < count ? b0 + FAM_PER_SLOT : count;
    for (int64_t i = b0 + threadIdx.x; i < b1; i += NT) {
        const FamilyRes v = in[i];
        for (int a = 0; a < 3; ++a) comp_add(t.S[a], c.S[a], v.m[a]);
        comp_add(t.L, c.L, v.ent);
        comp_add(t.P, c.P, v.p);
        t.gap = fmax(t.gap, v.gap);
        t.nu_cnt += v.nu;
        t.count += 1;
        if (v.x != 0) {
            for (int a = 0; a < 3; ++a) {
                comp_add(t.Snz[a], c.Snz[a], v.m[a]);
                comp_add(t.Q[a], c.Q[a], v.m[a] * v.m[a]);
            }
        }
    }
    fold_comp(t, c);
    sh[threadIdx.x] = t;
    __syncthreads();
    for (int h = NT / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) add_sums(sh[threadIdx.x], sh[threadIdx.x + h]);
        __syncthreads();
    }
    if (threadIdx.x == 0) out[blockIdx.x] = sh[0];
}

__global__ void __launch_bounds__(256)
k_reduce_sweep(const SweepSums* __restrict__ in, int64_t count, SweepSums* __restrict__ out) {
    constexpr int NT = 256;
    __shared__ SweepSums sh[NT];
    SweepSums t;
    zero_sums(t);
    SweepComp c;
    zero_comp(c);
    for (int64_t i = threadIdx.x; i < count; i += NT) {
        const SweepSums v = in[i];
        for (int a = 0; a < 3; ++a) {
            comp_add(t.S[a], c.S[a], v.S[a]);
            comp_add(t.Snz[a], c.Snz[a], v.Snz[a]);
            comp_add(t.Q[a], c.Q[a], v.Q[a]);
        }
        comp_add(t.L, c.L, v.L);
        comp_add(t.P, c.P, v.P);
        t.gap = fmax(t.gap, v.gap);
        t.nu_cnt += v.nu_cnt;
        t.count += v.count;
    }
    fold_comp(t, c);
    sh[threadIdx.x] = t;
    __syncthreads();
    for (int h = NT / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) add_sums(sh[threadIdx.x], sh[threadIdx.x + h]);
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

// Launch with optional timing events attached to the dispatch itself (sampled
// launches only; the others are plain launches, which graph capture records).
#define PW_LAUNCH(TM, KC, NB, KERNEL, GRID, BLOCK, ST, ...)                                      \
    do {                                                                                        \
        hipEvent_t ev0_ = nullptr, ev1_ = nullptr;                                              \
        const bool smp_ = (TM) != nullptr && (TM)->take((TM)->self, (KC), &ev0_, &ev1_);        \
        if (smp_) {                                                                             \
            hipExtLaunchKernelGGL(KERNEL, GRID, BLOCK, 0, ST, ev0_, ev1_, 0u, __VA_ARGS__);      \
            (TM)->commit((TM)->self, (KC), (NB), ev0_, ev1_);                                   \
        } else {                                                                                \
            hipLaunchKernelGGL(KERNEL, GRID, BLOCK, 0, ST, __VA_ARGS__);                        \
        }                                                                                       \
    } while (0)

// Tile shapes: first pass and column passes K = 12 (256 threads x 16 points,
// 35 KB (single) / 70 KB (double) of LDS); single-precision column passes use
// K = 13 (512 x 16, 70 KB) when that saves a pass; fused kernels K = n - 1.
constexpr int K_FIRST = 12;
constexpr int COL_RL = 4;
// points per thread of the next tile loaded while the two-tile reducing pass reduces the
// current one (16 of 64: 32 more VGPRs, no spills; 8 and 24 measured slower)
constexpr int COL15_PF = 16;
#ifndef COL15_LTL
#define COL15_LTL 9
#endif

template <typename R, int K, int MOM>
hipError_t launch_fused_k(const void* psi, const uint64_t* fpsi, int n, const uint64_t* xs, uint64_t x0, int nb, R eps,
                          FamilyRes* out, hipStream_t st, const LaunchTimer* tm) {
    constexpr int RL0 = K < 4 ? K : 4;
    constexpr int TL = K == 13 ? 9 : K - RL0;
    constexpr int RL = K - TL;
    PW_LAUNCH(tm, 0, nb, (k_fused<R, TL, RL, MOM>), dim3(nb), dim3(1 << TL), st, (const cx<R>*)psi, fpsi, n, xs, x0,
              eps, out);
    return hipGetLastError();
}

template <typename R, int MOM>
hipError_t launch_fused(const void* psi, const uint64_t* fpsi, int n, const uint64_t* xs, uint64_t x0, int nb, R eps,
                        FamilyRes* out, hipStream_t st, const LaunchTimer* tm) {
    switch (n - 1) {
#define PW_CASE(K) \
    case K: return launch_fused_k<R, K, MOM>(psi, fpsi, n, xs, x0, nb, eps, out, st, tm);
        PW_CASE(0) PW_CASE(1) PW_CASE(2) PW_CASE(3) PW_CASE(4) PW_CASE(5) PW_CASE(6)
        PW_CASE(7) PW_CASE(8) PW_CASE(9) PW_CASE(10) PW_CASE(11) PW_CASE(12)
#undef PW_CASE
        case 13:
            if constexpr (sizeof(R) == 4) return launch_fused_k<R, 13, MOM>(psi, fpsi, n, xs, x0, nb, eps, out, st, tm);
            return hipErrorInvalidValue;
        default: return hipErrorInvalidValue;
    }
}

template <typename R, int K, int MOM>
hipError_t launch_reduced_k(const void* rho, int na, uint64_t x0, int nb, R eps, FamilyRes* out, hipStream_t st) {
    constexpr int RL0 = K < 4 ? K : 4;
    constexpr int TL = K == 13 ? 9 : K - RL0;
    constexpr int RL = K - TL;
    hipLaunchKernelGGL((k_fused_reduced<R, TL, RL, MOM>), dim3(nb), dim3(1 << TL), 0, st, (const cx<R>*)rho, na, x0,
                       eps, out);
    return hipGetLastError();
}

template <typename R, int MOM>
hipError_t launch_reduced(const void* rho, int na, uint64_t x0, int nb, R eps, FamilyRes* out, hipStream_t st) {
    switch (na - 1) {
#define PW_CASE(K) \
    case K: return launch_reduced_k<R, K, MOM>(rho, na, x0, nb, eps, out, st);
        PW_CASE(0) PW_CASE(1) PW_CASE(2) PW_CASE(3) PW_CASE(4) PW_CASE(5) PW_CASE(6)
        PW_CASE(7) PW_CASE(8) PW_CASE(9) PW_CASE(10) PW_CASE(11) PW_CASE(12)
#undef PW_CASE
        case 13:
            if constexpr (sizeof(R) == 4) return launch_reduced_k<R, 13, MOM>(rho, na, x0, nb, eps, out, st);
            return hipErrorInvalidValue;
        default: return hipErrorInvalidValue;
    }
}

template <typename R, int TL, bool LAST, int MOM>
hipError_t launch_column_t(int s, dim3 grid, cx<R>* work, int n, int lo, const uint64_t* xs, uint64_t x0, R eps,
                           FamilyRes* parts, hipStream_t st, const LaunchTimer* tm) {
    const int kc = LAST ? 3 : 2;
    // the FP64 reducing pass exchanges real and imaginary parts in turn: half the LDS,
    // so that four workgroups per CU overlap their loads with the FP64 reductions
    constexpr bool SPLIT = LAST && sizeof(R) == 8;
    switch (s) {
#define PW_COL(S)                                                                                                    \
    case S:                                                                                                          \
        PW_LAUNCH(tm, kc, (int)grid.y, (k_column<R, TL, COL_RL, S, LAST, MOM, SPLIT, false>), grid, dim3(1 << TL), st, \
                  work, n, lo, xs, x0, eps, parts);                                                                  \
        return hipGetLastError();
        PW_COL(1) PW_COL(2) PW_COL(3) PW_COL(4) PW_COL(5) PW_COL(6) PW_COL(7) PW_COL(8) PW_COL(9)
#undef PW_COL
        default: return hipErrorInvalidValue;
    }
}

// Column pass over a 15-bit single-precision tile (1024 threads x 32 points, split
// LDS exchange): rows of 2^(15 - s) points, s = 9..12.
template <bool LAST, int MOM>
hipError_t launch_column15(int s, dim3 grid, cx<float>* work, int n, int lo, const uint64_t* xs, uint64_t x0,
                           float eps, FamilyRes* parts, hipStream_t st, const LaunchTimer* tm) {
    const int kc = LAST ? 3 : 2;
    switch (s) {
#define PW_COL15(S)                                                                                                \
    case S:                                                                                                        \
        if constexpr (LAST) {                                                                                      \
            if ((grid.x & 15u) == 0) {                                                                             \
                PW_LAUNCH(tm, kc, (int)grid.y,                                                                     \
                          (k_column<float, COL15_LTL, 15 - COL15_LTL, S, LAST, MOM, true, true, COL15_PF>),        \
                          dim3(grid.x / 2, grid.y), dim3(1 << COL15_LTL), st, work, n, lo, xs, x0, eps, parts);    \
            } else {                                                                                               \
                PW_LAUNCH(tm, kc, (int)grid.y, (k_column<float, COL15_LTL, 15 - COL15_LTL, S, LAST, MOM, true>),    \
                          grid, dim3(1 << COL15_LTL), st, work, n, lo, xs, x0, eps, parts);                        \
            }                                                                                                      \
        } else {                                                                                                   \
            PW_LAUNCH(tm, kc, (int)grid.y, (k_column<float, 10, 5, S, LAST, MOM, true>), grid, dim3(1024), st, work, \
                      n, lo, xs, x0, eps, parts);                                                                  \
        }                                                                                                          \
        return hipGetLastError();
        PW_COL15(9) PW_COL15(10) PW_COL15(11) PW_COL15(12)
#undef PW_COL15
        default: return hipErrorInvalidValue;
    }
}

template <typename R, bool LAST, int MOM>
hipError_t launch_column(int ktile, int s, int nh, int nb, cx<R>* work, int n, int lo, const uint64_t* xs,
                         uint64_t x0, R eps, FamilyRes* parts, hipStream_t st, const LaunchTimer* tm) {
    const dim3 grid(1u << (nh - ktile), nb);
    if constexpr (sizeof(R) == 4) {
        if (ktile == 13) return launch_column_t<R, 9, LAST, MOM>(s, grid, work, n, lo, xs, x0, eps, parts, st, tm);
        if (ktile == 15) return launch_column15<LAST, MOM>(s, grid, work, n, lo, xs, x0, eps, parts, st, tm);
    }
    if (ktile != 12) return hipErrorInvalidValue;
    return launch_column_t<R, 8, LAST, MOM>(s, grid, work, n, lo, xs, x0, eps, parts, st, tm);
}

template <int MOM>
hipError_t launch_fused_mfma(const void* psi, const uint64_t* fpsi, int n, const uint64_t* xs, uint64_t x0, int nb,
                             float eps, FamilyRes* out, hipStream_t st, const LaunchTimer* tm) {
    switch (n - 1) {
#define PW_MF(K, LB, LW)                                                                                           \
    case K:                                                                                                        \
        PW_LAUNCH(tm, 0, nb, (k_fused_mfma<LB, LW, MOM>), dim3(nb), dim3(64 << LW), st, (const cx<float>*)psi, fpsi, \
                  n, xs, x0, eps, out);                                                                            \
        return hipGetLastError();
        PW_MF(8, 0, 0) PW_MF(9, 1, 0) PW_MF(10, 2, 0) PW_MF(11, 2, 1) PW_MF(12, 2, 2) PW_MF(13, 3, 2)
#undef PW_MF
        default: return hipErrorInvalidValue;
    }
}

// First pass over nb families, with the tile-sharing groups where first_pass_group
// asks for them.
template <typename R, int TL, int RL, bool SPLIT>
void launch_first(const Plan& P, const void* psi, const uint64_t* fpsi, const uint64_t* xs, uint64_t x0, int nb,
                  void* work, hipStream_t st, const LaunchTimer* tm) {
    const uint32_t tiles = 1u << (P.nh - TL - RL);
    const int grp = first_pass_group(P, sizeof(R) == 8, nb);
    const uint32_t blocks = tiles * (uint32_t)((nb + grp - 1) / grp * grp);
    if (grp == 128)
        PW_LAUNCH(tm, 1, nb, (k_first<R, TL, RL, SPLIT, false, 128>), dim3(blocks), dim3(1 << TL), st,
                  (const cx<R>*)psi, fpsi, P.n, xs, x0, (cx<R>*)work, nb);
    else if (grp == 64)
        PW_LAUNCH(tm, 1, nb, (k_first<R, TL, RL, SPLIT, false, 64>), dim3(blocks), dim3(1 << TL), st,
                  (const cx<R>*)psi, fpsi, P.n, xs, x0, (cx<R>*)work, nb);
    else if (grp == 32)
        PW_LAUNCH(tm, 1, nb, (k_first<R, TL, RL, SPLIT, false, 32>), dim3(blocks), dim3(1 << TL), st,
                  (const cx<R>*)psi, fpsi, P.n, xs, x0, (cx<R>*)work, nb);
    else if (grp == 16)
        PW_LAUNCH(tm, 1, nb, (k_first<R, TL, RL, SPLIT, false, 16>), dim3(blocks), dim3(1 << TL), st,
                  (const cx<R>*)psi, fpsi, P.n, xs, x0, (cx<R>*)work, nb);
    else if (grp == 8)
        PW_LAUNCH(tm, 1, nb, (k_first<R, TL, RL, SPLIT, false, 8>), dim3(blocks), dim3(1 << TL), st,
                  (const cx<R>*)psi, fpsi, P.n, xs, x0, (cx<R>*)work, nb);
    else if (grp == 4)
        PW_LAUNCH(tm, 1, nb, (k_first<R, TL, RL, SPLIT, false, 4>), dim3(blocks), dim3(1 << TL), st,
                  (const cx<R>*)psi, fpsi, P.n, xs, x0, (cx<R>*)work, nb);
    else if (grp == 2)
        PW_LAUNCH(tm, 1, nb, (k_first<R, TL, RL, SPLIT, false, 2>), dim3(blocks), dim3(1 << TL), st,
                  (const cx<R>*)psi, fpsi, P.n, xs, x0, (cx<R>*)work, nb);
    else
        PW_LAUNCH(tm, 1, nb, (k_first<R, TL, RL, SPLIT>), dim3(tiles, nb), dim3(1 << TL), st, (const cx<R>*)psi, fpsi,
                  P.n, xs, x0, (cx<R>*)work, nb);
}

template <typename R, int MOM>
hipError_t eval_batch_t(const Plan& P, const void* psi, const uint64_t* fpsi, const uint64_t* xs, uint64_t x0, int nb,
                        double eps, void* work, FamilyRes* parts, FamilyRes* out, hipStream_t st,
                        const LaunchTimer* tm, bool finalize) {
    if (nb <= 0) return hipSuccess;
    if (fpsi && !xs) return hipErrorInvalidValue;   // per-family states come with a list
    const R e = (R)eps;
    if constexpr (sizeof(R) == 4) {
        if (P.fused && P.mfma && P.nh >= 8) return launch_fused_mfma<MOM>(psi, fpsi, P.n, xs, x0, nb, e, out, st, tm);
    }
    if (P.fused) return launch_fused<R, MOM>(psi, fpsi, P.n, xs, x0, nb, e, out, st, tm);
    const uint32_t tiles = 1u << (P.nh - P.k1);
    if constexpr (sizeof(R) == 4) {
        if (P.mfma) {
            if (P.k1 != K_FIRST) return hipErrorInvalidValue;
            PW_LAUNCH(tm, 1, nb, k_first_mfma, dim3(tiles, nb), dim3(256), st, (const cx<float>*)psi, fpsi, P.n, xs,
                      x0, (cx<float>*)work);
            goto first_done;
        }
        if (P.k1 == 15) {
            launch_first<float, 10, 5, true>(P, psi, fpsi, xs, x0, nb, work, st, tm);
            goto first_done;
        }
    }
    if (!xs && x0 >= (1ull << K_FIRST) && (x0 >> 8) == ((x0 + nb - 1) >> 8) && (x0 % nb) == 0) {
        // a run of consecutive families inside one 256-aligned block: share the state tiles,
        // up to 16 families per workgroup while the grid keeps >= 512 workgroups (two per CU;
        // longer runs measured faster than more, shorter workgroups)
        int fam = 1;
        while (fam < 16 && (nb % (2 * fam)) == 0 && (uint64_t)tiles * (nb / (2 * fam)) >= 512) fam *= 2;
        PW_LAUNCH(tm, 1, nb, (k_first_shared<R, 8, 4>), dim3(tiles, nb / fam), dim3(256), st, (const cx<R>*)psi, P.n,
                  x0, fam, (cx<R>*)work);
    } else {
        launch_first<R, 8, 4, false>(P, psi, fpsi, xs, x0, nb, work, st, tm);
    }
first_done:
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
    for (int i = 0; i < P.npass; ++i) {
        const bool last = i + 1 == P.npass;
        err = last ? launch_column<R, true, MOM>(P.ktile, P.s[i], P.nh, nb, (cx<R>*)work, P.n, P.lo[i], xs, x0, e,
                                                 parts, st, tm)
                   : launch_column<R, false, 2>(P.ktile, P.s[i], P.nh, nb, (cx<R>*)work, P.n, P.lo[i], xs, x0, e,
                                                parts, st, tm);
        if (err != hipSuccess) return err;
    }
    if (!finalize) return hipSuccess;
    launch_finalize<MOM>(parts, P.blocks_last, P.n, nb, out, st);
    return hipGetLastError();
}

template <typename R, int K>
hipError_t launch_store_k(const void* psi, int n, uint64_t x, void* G, hipStream_t st) {
    constexpr int RL0 = K < 4 ? K : 4;
    constexpr int TL = K == 13 ? 9 : K - RL0;
    constexpr int RL = K - TL;
    hipLaunchKernelGGL((k_fused_store<R, TL, RL>), dim3(1), dim3(1 << TL), 0, st, (const cx<R>*)psi, n, x, (cx<R>*)G);
    return hipGetLastError();
}

template <typename R>
hipError_t transform_one_t(const Plan& P, const void* psi, uint64_t x, void* work, hipStream_t st) {
    const int nh = P.nh;
    if (P.fused) {
        // the single-workgroup transform, written out instead of reduced
        switch (nh) {
#define PW_CASE(K) \
    case K: return launch_store_k<R, K>(psi, P.n, x, work, st);
            PW_CASE(0) PW_CASE(1) PW_CASE(2) PW_CASE(3) PW_CASE(4) PW_CASE(5) PW_CASE(6)
            PW_CASE(7) PW_CASE(8) PW_CASE(9) PW_CASE(10) PW_CASE(11) PW_CASE(12)
#undef PW_CASE
            case 13:
                if constexpr (sizeof(R) == 4) return launch_store_k<R, 13>(psi, P.n, x, work, st);
                return hipErrorInvalidValue;
            default: return hipErrorInvalidValue;
        }
    }
    // the multi-pass schedule without the final reduction
    if (nh <= K_FIRST) return hipErrorInvalidValue;
    bool done = false;
    if constexpr (sizeof(R) == 4) {
        if (P.k1 == 15) {
            hipLaunchKernelGGL((k_first<float, 10, 5, true>), dim3(1u << (nh - 15), 1), dim3(1024), 0, st,
                               (const cx<float>*)psi, (const uint64_t*)nullptr, P.n, (const uint64_t*)nullptr, x,
                               (cx<float>*)work, 1);
            done = true;
        }
    }
    if (!done)
        hipLaunchKernelGGL((k_first<R, 8, 4>), dim3(1u << (nh - K_FIRST), 1), dim3(256), 0, st, (const cx<R>*)psi,
                           (const uint64_t*)nullptr, P.n, (const uint64_t*)nullptr, x, (cx<R>*)work, 1);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
    for (int i = 0; i < P.npass; ++i) {
        err = launch_column<R, false, 2>(P.ktile, P.s[i], nh, 1, (cx<R>*)work, P.n, P.lo[i], (const uint64_t*)nullptr,
                                         x, (R)0, (FamilyRes*)nullptr, st, nullptr);
        if (err != hipSuccess) return err;
    }
    return hipSuccess;
}

}  // namespace

namespace {
Plan make_plan_impl(int n, bool dbl, bool allow15);
}

Plan make_plan(int n, bool dbl) { return make_plan_impl(n, dbl, true); }

Plan make_plan_sched(int n, bool dbl, const Schedule& sc, bool* honoured) {
    Plan P = make_plan_impl(n, dbl, true);
    bool ok = true;
    if (sc.group < 0 || sc.group > GROUP_MAX || (sc.group & (sc.group - 1)) != 0) ok = false;
    if (!P.fused && ok && (sc.first_bits != 0 || sc.column_tile_bits != 0)) {
        const int nh = n - 1;
        int k1 = sc.first_bits ? sc.first_bits : P.k1;
        if (k1 == 15) {
            // 15-bit first pass, one column pass of s = n - 1 - 15 bits
            const int sbits = nh - 15;
            int kt = sc.column_tile_bits ? sc.column_tile_bits : (sbits <= 8 ? 12 : 15);
            const bool fits = (kt == 12 && sbits <= 8) || (kt == 13 && sbits <= 9) || (kt == 15 && sbits >= 9);
            if (dbl || sbits < 1 || sbits > 12 || !fits) {
                ok = false;
            } else {
                P.k1 = 15;
                P.npass = 1;
                P.lo[0] = 15;
                P.s[0] = sbits;
                P.ktile = kt;
                P.blocks_last = 1 << (nh - kt);
            }
        } else if (k1 == 12) {
            const int kt = sc.column_tile_bits ? sc.column_tile_bits : (dbl ? 12 : 0);
            if (kt != 0 && kt != 12 && !(kt == 13 && !dbl)) {
                ok = false;
            } else {
                const Plan D = make_plan_impl(n, dbl, false);
                P = D;
                if (kt != 0 && kt != D.ktile) {
                    // the other column tile: re-split the remaining bits for it
                    const int smax = kt == 13 ? 9 : (dbl ? 9 : 8);
                    const int rem = nh - K_FIRST;
                    const int np = (rem + smax - 1) / smax;
                    if (np > 4) {
                        ok = false;
                    } else {
                        P.ktile = kt;
                        P.npass = np;
                        int lo = K_FIRST;
                        for (int i = 0; i < np; ++i) {
                            const int left = nh - lo;
                            const int sb = (left + (np - i) - 1) / (np - i);
                            P.lo[i] = lo;
                            P.s[i] = sb;
                            lo += sb;
                        }
                        P.blocks_last = 1 << (nh - kt);
                    }
                }
            }
        } else {
            ok = false;
        }
    }
    if (!ok) {
        if (honoured) *honoured = false;
        return make_plan_impl(n, dbl, true);
    }
    P.grp_req = P.fused ? 0 : sc.group;
    if (honoured) *honoured = true;
    return P;
}

Plan make_plan_bf16x2(int n) {
    Plan P = make_plan_impl(n, false, false);
    P.mfma = true;
    return P;
}

namespace {
Plan make_plan_impl(int n, bool dbl, bool allow15) {
    Plan P{};
    P.n = n;
    P.nh = n - 1;
    const int fmax = dbl ? 12 : 13;
    if (P.nh <= fmax) {
        P.fused = true;
        P.k1 = P.nh;
        P.npass = 0;
        P.blocks_last = 1;
        return P;
    }
    P.fused = false;
    if (!dbl && allow15 && P.nh >= 22 && P.nh <= 27) {
        // single precision, n = 23..28: a 15-bit first pass leaves one column pass
        P.k1 = 15;
        P.npass = 1;
        P.lo[0] = 15;
        P.s[0] = P.nh - 15;
        P.ktile = P.s[0] <= 8 ? 12 : 15;
        P.blocks_last = 1 << (P.nh - P.ktile);
        return P;
    }
    P.k1 = K_FIRST;
    const int rem = P.nh - K_FIRST;
    // column tiles of 2^ktile points with rows of >= 128 bytes: s <= ktile - 4 (single),
    // ktile - 3 (double); single precision takes 13-bit tiles when that saves a pass
    int ktile = 12;
    int smax = dbl ? 9 : 8;
    if (!dbl && (rem + 7) / 8 > (rem + 8) / 9) {
        ktile = 13;
        smax = 9;
    }
    P.ktile = ktile;
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
}  // namespace

hipError_t eval_batch(const Plan& P, bool dbl, int max_alpha, const void* psi, const uint64_t* xs, uint64_t x0,
                      int nb, double eps, void* work, FamilyRes* parts, FamilyRes* out, hipStream_t st,
                      const LaunchTimer* tm, bool finalize, const uint64_t* fpsi) {
    if (dbl)
        return max_alpha >= 4
                   ? eval_batch_t<double, 4>(P, psi, fpsi, xs, x0, nb, eps, work, parts, out, st, tm, finalize)
                   : eval_batch_t<double, 2>(P, psi, fpsi, xs, x0, nb, eps, work, parts, out, st, tm, finalize);
    return max_alpha >= 4 ? eval_batch_t<float, 4>(P, psi, fpsi, xs, x0, nb, eps, work, parts, out, st, tm, finalize)
                          : eval_batch_t<float, 2>(P, psi, fpsi, xs, x0, nb, eps, work, parts, out, st, tm, finalize);
}

hipError_t finalize_families(const Plan& P, int max_alpha, const FamilyRes* parts, int64_t nfam, FamilyRes* out,
                             hipStream_t st) {
    if (P.fused || nfam <= 0) return hipSuccess;
    if (nfam > 0x7fffffff) return hipErrorInvalidValue;
    if (max_alpha >= 4)
        launch_finalize<4>(parts, P.blocks_last, P.n, nfam, out, st);
    else
        launch_finalize<2>(parts, P.blocks_last, P.n, nfam, out, st);
    return hipGetLastError();
}

hipError_t reduced_density(bool dbl, const void* psi, int n, int na, void* rho, hipStream_t st,
                           const LaunchTimer* tm) {
    const unsigned tiles = (unsigned)(((1u << na) + 63) / 64);
    if (dbl)
        PW_LAUNCH(tm, 4, 1, k_rho<double>, dim3(tiles, tiles), dim3(256), st, (const cx<double>*)psi, na, n - na,
                  (cx<double>*)rho);
    else
        PW_LAUNCH(tm, 4, 1, k_rho<float>, dim3(tiles, tiles), dim3(256), st, (const cx<float>*)psi, na, n - na,
                  (cx<float>*)rho);
    return hipGetLastError();
}

// Families of the reduced state too large for one workgroup: the first pass reads h rows
// of D, then the column passes and the per-family finalisation of the state path.
template <typename R, int MOM>
hipError_t eval_reduced_mp_t(const Plan& P, const void* D, uint64_t x0, int nb, double eps, void* work,
                             FamilyRes* parts, FamilyRes* out, hipStream_t st) {
    if (P.fused || P.k1 != K_FIRST) return hipErrorInvalidValue;
    const R e = (R)eps;
    const uint32_t tiles = 1u << (P.nh - P.k1);
    hipLaunchKernelGGL((k_first<R, 8, 4, false, true>), dim3(tiles, nb), dim3(256), 0, st, (const cx<R>*)D,
                       (const uint64_t*)nullptr, P.n, (const uint64_t*)nullptr, x0, (cx<R>*)work, nb);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
    for (int i = 0; i < P.npass; ++i) {
        const bool last = i + 1 == P.npass;
        err = last ? launch_column<R, true, MOM>(P.ktile, P.s[i], P.nh, nb, (cx<R>*)work, P.n, P.lo[i], nullptr, x0,
                                                 e, parts, st, nullptr)
                   : launch_column<R, false, 2>(P.ktile, P.s[i], P.nh, nb, (cx<R>*)work, P.n, P.lo[i], nullptr, x0, e,
                                                parts, st, nullptr);
        if (err != hipSuccess) return err;
    }
    launch_finalize<MOM>(parts, P.blocks_last, P.n, nb, out, st);
    return hipGetLastError();
}

hipError_t eval_reduced_batch(bool dbl, int max_alpha, const void* rho, int na, uint64_t x0, int nb, double eps,
                              void* work, FamilyRes* parts, FamilyRes* out, hipStream_t st) {
    if (nb <= 0) return hipSuccess;
    const Plan P = make_plan(na, dbl);
    if (!P.fused) {
        if (dbl)
            return max_alpha >= 4 ? eval_reduced_mp_t<double, 4>(P, rho, x0, nb, eps, work, parts, out, st)
                                  : eval_reduced_mp_t<double, 2>(P, rho, x0, nb, eps, work, parts, out, st);
        return max_alpha >= 4 ? eval_reduced_mp_t<float, 4>(P, rho, x0, nb, eps, work, parts, out, st)
                              : eval_reduced_mp_t<float, 2>(P, rho, x0, nb, eps, work, parts, out, st);
    }
    if (dbl)
        return max_alpha >= 4 ? launch_reduced<double, 4>(rho, na, x0, nb, eps, out, st)
                              : launch_reduced<double, 2>(rho, na, x0, nb, eps, out, st);
    return max_alpha >= 4 ? launch_reduced<float, 4>(rho, na, x0, nb, (float)eps, out, st)
                          : launch_reduced<float, 2>(rho, na, x0, nb, (float)eps, out, st);
}

int first_pass_group(const Plan& P, bool dbl, int nb) {
    if (P.grp_req > 0) {
        // a schedule's group, within the launch and the numbering's need of 8 tiles
        if (P.fused || P.mfma || P.nh - P.k1 < 3) return 1;
        int g = 1;
        while (g * 2 <= P.grp_req && g * 2 <= nb) g *= 2;
        return g;
    }
    // states of 16 MiB and more (measured: 4-21 % less time per family from 16 MiB to
    // 8 GiB); at least 8 tiles per family, which the grouped numbering needs
    if (P.fused || P.mfma || P.nh - P.k1 < 3 || ((size_t)(dbl ? 16 : 8) << P.n) < ((size_t)16 << 20)) return 1;
    // the whole launch as one group, up to 128 families (measured at n = 28, per family of the
    // first pass: launches of 64 in groups of 4: 870 us, 8: 806, 16: 780 (whole path), 32: 436,
    // 64: 416; launches of 128 in groups of 64: 428, of 128: 404; n = 30: 4156 -> 4094 us from
    // groups of four to eight)
    int g = 1;
    while (g * 2 <= nb && g * 2 <= GROUP_MAX) g *= 2;
    return g;
}

hipError_t sort_by_top_bit(const uint64_t* xs, int n, int nx, uint64_t* xs_sorted, uint32_t* perm, hipStream_t st) {
    if (nx <= 0) return hipSuccess;
    if (nx > SORT_MAX || n < 1 || n > 32) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_sort_top, dim3(1), dim3(64), 0, st, xs, n, nx, xs_sorted, perm);
    return hipGetLastError();
}

hipError_t scatter_results(const FamilyRes* in, const uint32_t* perm, int nx, FamilyRes* out, hipStream_t st) {
    if (nx <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_scatter_res, dim3((unsigned)((nx + 255) / 256)), dim3(256), 0, st, in, perm, nx, out);
    return hipGetLastError();
}

hipError_t reduce_families(const FamilyRes* in, int64_t count, SweepSums* out, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_reduce_fam, dim3((unsigned)reduce_families_slots(count)), dim3(256), 0, st, in, count, out);
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
