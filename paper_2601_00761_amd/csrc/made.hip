// Learned proposal over X-bitstrings: a masked autoregressive network (MADE,
// Germain et al. 2015) N -> h -> h -> N with ReLU hidden layers, Bernoulli outputs
// and direct input->output connections, in FP32.  Hidden unit k has degree
// deg(k) = (k mod (N-1)) + 1 and bit i of x is input i (degree i+1), so output i,
// the logit of P(x_i = 1 | x_0..x_{i-1}), sees bits j < i only.  Kernels: forward
// (activations + log q in FP64), backward (per-sample error signals), weight
// gradients (fixed-order sums over the minibatch), Adam, and the autoregressive
// sampler, which recomputes the same forward code for every prefix so that the
// logits it samples from are bitwise those that the log-density kernel returns.
//
// Parameter layout (floats): W1T[n*h] (i*h + k), b1[h], W2T[h*h] (kk*h + k), b2[h],
// W3T[h*n] (kk*n + i), b3[n], AT[n*n] (j*n + i).
#include "common.h"
#include "philox.h"
#include <math.h>

namespace pw {

MadeDims made_dims(int n, int h) {
    MadeDims D{};
    D.n = n;
    D.h = h;
    size_t o = 0;
    D.oW1 = o;
    o += (size_t)n * h;
    D.ob1 = o;
    o += h;
    D.oW2 = o;
    o += (size_t)h * h;
    D.ob2 = o;
    o += h;
    D.oW3 = o;
    o += (size_t)h * n;
    D.ob3 = o;
    o += n;
    D.oA = o;
    o += (size_t)n * n;
    D.total = o;
    return D;
}

namespace {

__device__ __forceinline__ int deg(int k, int n) { return (k % (n - 1)) + 1; }

// Hidden activations of this thread's units for input bits xin (in LDS).
template <int H>
__device__ __forceinline__ void hidden(const float* __restrict__ P, const MadeDims& D, const float* xin, float* h1s,
                                       float* h2s, float& h1, float& h2) {
    const int n = D.n, k = threadIdx.x;
    const int dk = deg(k, n);
    float a = P[D.ob1 + k];
    for (int i = 0; i < n; ++i) {
        const float m = (i + 1 <= dk) ? 1.f : 0.f;
        a = fmaf(P[D.oW1 + (size_t)i * H + k] * m, xin[i], a);
    }
    h1 = fmaxf(a, 0.f);
    h1s[k] = h1;
    __syncthreads();
    a = P[D.ob2 + k];
    for (int kk = 0; kk < H; ++kk) {
        const float m = (deg(kk, n) <= dk) ? 1.f : 0.f;
        a = fmaf(P[D.oW2 + (size_t)kk * H + k] * m, h1s[kk], a);
    }
    h2 = fmaxf(a, 0.f);
    h2s[k] = h2;
    __syncthreads();
}

// Logit of output i (sequential sum over the hidden units, then the direct terms).
template <int H>
__device__ __forceinline__ float out_logit(const float* __restrict__ P, const MadeDims& D, int i, const float* h2s,
                                           const float* xin) {
    const int n = D.n;
    float o = P[D.ob3 + i];
    for (int kk = 0; kk < H; ++kk) {
        const float m = (deg(kk, n) <= i) ? 1.f : 0.f;
        o = fmaf(P[D.oW3 + (size_t)kk * n + i] * m, h2s[kk], o);
    }
    for (int j = 0; j < i; ++j) o = fmaf(P[D.oA + (size_t)j * n + i], xin[j], o);
    return o;
}

// log s(o) = -softplus(-o), stable for large |o|.
__device__ __forceinline__ double log_sig(double o) { return o >= 0.0 ? -log1p(exp(-o)) : o - log1p(exp(o)); }

template <int H>
__global__ void __launch_bounds__(H)
k_made_fwd(const float* __restrict__ P, MadeDims D, const uint64_t* __restrict__ xs, const int* __restrict__ perm,
           float* __restrict__ H1, float* __restrict__ H2, float* __restrict__ O, double* __restrict__ logq) {
    __shared__ float xin[64], h1s[H], h2s[H];
    const int b = blockIdx.x, k = threadIdx.x, n = D.n;
    const uint64_t x = xs[perm ? perm[b] : b];
    if (k < 64) xin[k] = (k < n && ((x >> k) & 1ull)) ? 1.f : 0.f;
    __syncthreads();
    float h1, h2;
    hidden<H>(P, D, xin, h1s, h2s, h1, h2);
    if (H1) H1[(size_t)b * H + k] = h1;
    if (H2) H2[(size_t)b * H + k] = h2;
    double ll = 0.0;
    if (k < n) {
        const float o = out_logit<H>(P, D, k, h2s, xin);
        if (O) O[(size_t)b * n + k] = o;
        ll = xin[k] > 0.5f ? log_sig((double)o) : log_sig(-(double)o);
    }
    // outputs live in wave 0 (n <= 32): fixed-order shuffle sum
    if (k < 64) {
        for (int off = 32; off > 0; off >>= 1) ll += __shfl_xor(ll, off);
        if (k == 0 && logq) logq[b] = ll;
    }
}

// Per-sample error signals for the weighted NLL: dO = w_b/W (s(o) - x),
// G2 = relu'(a2) * (W3 M3)^T dO, G1 = relu'(a1) * (W2 M2)^T G2.
template <int H>
__global__ void __launch_bounds__(H)
k_made_bwd(const float* __restrict__ P, MadeDims D, const uint64_t* __restrict__ xs, const int* __restrict__ perm,
           const float* __restrict__ w, float invW, const float* __restrict__ H1, const float* __restrict__ H2,
           const float* __restrict__ O, float* __restrict__ dO, float* __restrict__ G1, float* __restrict__ G2) {
    __shared__ float dos[64], g2s[H];
    const int b = blockIdx.x, k = threadIdx.x, n = D.n;
    const int src = perm ? perm[b] : b;
    const uint64_t x = xs[src];
    if (k < 64) {
        float d = 0.f;
        if (k < n) {
            const float o = O[(size_t)b * n + k];
            const float s = 1.f / (1.f + expf(-o));
            const float xb = ((x >> k) & 1ull) ? 1.f : 0.f;
            d = w[src] * invW * (s - xb);
            dO[(size_t)b * n + k] = d;
        }
        dos[k] = d;
    }
    __syncthreads();
    const int dk = deg(k, n);
    float g2 = 0.f;
    for (int i = 0; i < n; ++i) {
        const float m = (dk <= i) ? 1.f : 0.f;
        g2 = fmaf(P[D.oW3 + (size_t)k * n + i] * m, dos[i], g2);
    }
    g2 = H2[(size_t)b * H + k] > 0.f ? g2 : 0.f;
    g2s[k] = g2;
    G2[(size_t)b * H + k] = g2;
    __syncthreads();
    float g1 = 0.f;
    for (int k2 = 0; k2 < H; ++k2) {
        const float m = (deg(k2, n) >= dk) ? 1.f : 0.f;
        g1 = fmaf(P[D.oW2 + (size_t)k * H + k2] * m, g2s[k2], g1);
    }
    G1[(size_t)b * H + k] = H1[(size_t)b * H + k] > 0.f ? g1 : 0.f;
}

// Weight gradients: one thread per parameter, a fixed-order sum over the minibatch.
template <int H>
__global__ void __launch_bounds__(256)
k_made_wgrad(MadeDims D, const uint64_t* __restrict__ xs, const int* __restrict__ perm, int B,
             const float* __restrict__ dO, const float* __restrict__ G1, const float* __restrict__ G2,
             const float* __restrict__ H1, const float* __restrict__ H2, float* __restrict__ grad) {
    const size_t p = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (p >= D.total) return;
    const int n = D.n;
    float s = 0.f;
    if (p < D.ob1) {                               // W1T[i*H + k]
        const int i = (int)(p / H), k = (int)(p % H);
        if (i + 1 <= deg(k, n))
            for (int b = 0; b < B; ++b) {
                const uint64_t x = xs[perm ? perm[b] : b];
                if ((x >> i) & 1ull) s += G1[(size_t)b * H + k];
            }
    } else if (p < D.oW2) {                        // b1[k]
        const int k = (int)(p - D.ob1);
        for (int b = 0; b < B; ++b) s += G1[(size_t)b * H + k];
    } else if (p < D.ob2) {                        // W2T[kk*H + k]
        const size_t q = p - D.oW2;
        const int kk = (int)(q / H), k = (int)(q % H);
        if (deg(kk, n) <= deg(k, n))
            for (int b = 0; b < B; ++b) s = fmaf(G2[(size_t)b * H + k], H1[(size_t)b * H + kk], s);
    } else if (p < D.oW3) {                        // b2[k]
        const int k = (int)(p - D.ob2);
        for (int b = 0; b < B; ++b) s += G2[(size_t)b * H + k];
    } else if (p < D.ob3) {                        // W3T[kk*n + i]
        const size_t q = p - D.oW3;
        const int kk = (int)(q / n), i = (int)(q % n);
        if (deg(kk, n) <= i)
            for (int b = 0; b < B; ++b) s = fmaf(dO[(size_t)b * n + i], H2[(size_t)b * H + kk], s);
    } else if (p < D.oA) {                         // b3[i]
        const int i = (int)(p - D.ob3);
        for (int b = 0; b < B; ++b) s += dO[(size_t)b * n + i];
    } else {                                       // AT[j*n + i], j < i
        const size_t q = p - D.oA;
        const int j = (int)(q / n), i = (int)(q % n);
        if (j < i)
            for (int b = 0; b < B; ++b) {
                const uint64_t x = xs[perm ? perm[b] : b];
                if ((x >> j) & 1ull) s += dO[(size_t)b * n + i];
            }
    }
    grad[p] = s;
}

__global__ void __launch_bounds__(256)
k_adam(float* __restrict__ P, const float* __restrict__ g, float* __restrict__ m, float* __restrict__ v, size_t count,
       float lr, float b1, float b2, float eps, float c1, float c2) {
    const size_t p = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (p >= count) return;
    const float gp = g[p];
    const float mp = b1 * m[p] + (1.f - b1) * gp;
    const float vp = b2 * v[p] + (1.f - b2) * gp * gp;
    m[p] = mp;
    v[p] = vp;
    P[p] -= lr * (mp / c1) / (sqrtf(vp / c2) + eps);
}

// Autoregressive draws conditioned on x != 0: for bit j the forward pass runs on the
// prefix (later bits 0, which the masks ignore) and u = (W0 >> 40) 2^-24 from
// Philox(ctr = (offset+i, attempt*64 + j, MADE), key = seed) sets x_j = [u < s(o_j)].
template <int H>
__global__ void __launch_bounds__(H)
k_made_sample(const float* __restrict__ P, MadeDims D, uint64_t seed, uint64_t offset, uint64_t* __restrict__ xs) {
    __shared__ float xin[64], h1s[H], h2s[H];
    __shared__ uint64_t xsh;
    const int k = threadIdx.x, n = D.n;
    const uint64_t g = offset + blockIdx.x;
    uint64_t x = 0;
    for (int a = 0; a < 64; ++a) {
        if (k < 64) xin[k] = 0.f;
        if (k == 0) xsh = 0;
        __syncthreads();
        for (int j = 0; j < n; ++j) {
            float h1, h2;
            hidden<H>(P, D, xin, h1s, h2s, h1, h2);
            if (k == 0) {
                const float o = out_logit<H>(P, D, j, h2s, xin);
                const float p1 = 1.f / (1.f + expf(-o));
                uint64_t W0, W1;
                philox_words(seed, g, (uint32_t)(a * 64 + j), STREAM_MADE, W0, W1);
                const float u = (float)(W0 >> 40) * 0x1.0p-24f;
                if (u < p1) {
                    xin[j] = 1.f;
                    xsh |= 1ull << j;
                }
            }
            __syncthreads();
        }
        x = xsh;
        __syncthreads();
        if (x != 0) break;
    }
    if (k == 0) xs[blockIdx.x] = x;
}

template <int H> struct MadeH {};

}  // namespace

#define PW_MADE_DISPATCH(HVAL, CALL) \
    switch (HVAL) {                  \
        case 64: { constexpr int H = 64; CALL; } break;   \
        case 128: { constexpr int H = 128; CALL; } break; \
        case 256: { constexpr int H = 256; CALL; } break; \
        default: return hipErrorInvalidValue;            \
    }

hipError_t made_forward(const MadeDims& D, const float* P, const uint64_t* xs, const int* perm, int B, float* H1,
                        float* H2, float* O, double* logq, hipStream_t st) {
    if (B <= 0) return hipSuccess;
    PW_MADE_DISPATCH(D.h, hipLaunchKernelGGL(k_made_fwd<H>, dim3(B), dim3(H), 0, st, P, D, xs, perm, H1, H2, O, logq));
    return hipGetLastError();
}

hipError_t made_backward(const MadeDims& D, const float* P, const uint64_t* xs, const int* perm, const float* w,
                         float invW, int B, const float* H1, const float* H2, const float* O, float* dO, float* G1,
                         float* G2, hipStream_t st) {
    if (B <= 0) return hipSuccess;
    PW_MADE_DISPATCH(D.h, hipLaunchKernelGGL(k_made_bwd<H>, dim3(B), dim3(H), 0, st, P, D, xs, perm, w, invW, H1, H2,
                                             O, dO, G1, G2));
    return hipGetLastError();
}

hipError_t made_wgrad(const MadeDims& D, const uint64_t* xs, const int* perm, int B, const float* dO, const float* G1,
                      const float* G2, const float* H1, const float* H2, float* grad, hipStream_t st) {
    const unsigned blocks = (unsigned)((D.total + 255) / 256);
    PW_MADE_DISPATCH(D.h, hipLaunchKernelGGL(k_made_wgrad<H>, dim3(blocks), dim3(256), 0, st, D, xs, perm, B, dO, G1,
                                             G2, H1, H2, grad));
    return hipGetLastError();
}

hipError_t made_adam(float* P, const float* g, float* m, float* v, size_t count, float lr, float b1, float b2,
                     float eps, int t, hipStream_t st) {
    const float c1 = 1.f - powf(b1, (float)t), c2 = 1.f - powf(b2, (float)t);
    hipLaunchKernelGGL(k_adam, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, P, g, m, v, count, lr, b1, b2,
                       eps, c1, c2);
    return hipGetLastError();
}

hipError_t made_sample(const MadeDims& D, const float* P, uint64_t seed, uint64_t offset, int64_t count, uint64_t* xs,
                       hipStream_t st) {
    if (count <= 0) return hipSuccess;
    PW_MADE_DISPATCH(D.h, hipLaunchKernelGGL(k_made_sample<H>, dim3((unsigned)count), dim3(H), 0, st, P, D, seed,
                                             offset, xs));
    return hipGetLastError();
}

}  // namespace pw
