// Internal declarations shared by the HIP translation units of libpauliwht.
// Not part of the public C ABI (that is include/pauliwht.h).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include <string>
#include <vector>

namespace pw {

template <typename R>
struct __align__(2 * sizeof(R)) cx {
    R re, im;
};

// Per-family accumulators, FP64.  One per workgroup of the final transform pass,
// then one per family after the fixed-order finalize.  Layout matches pw_xres
// from the public header (x, p, ent, m[3], gap, nu).
struct FamilyRes {
    uint64_t x;
    double p;       // sum |F|^2 (scaled by 2^-n at finalize)
    double ent;     // sum |F|^2 log2 |F|^2
    double m[3];    // sum |F|^{2a}, a = 2, 3, 4 (scaled by 2^-na at finalize)
    double gap;     // max |F| below 1 - eps, -1 if none
    uint64_t nu;    // count of ||F| - 1| < eps
};
static_assert(sizeof(FamilyRes) == 64, "FamilyRes layout");

// Sums over a set of families (exact sweep, batch level).
struct SweepSums {
    double S[3];
    double L;
    double P;
    double gap;
    uint64_t nu_cnt;
    uint64_t count;
    double Snz[3];  // sum over x != 0 of m_{alpha;x}
    double Q[3];    // sum over x != 0 of m_{alpha;x}^2 (spread of the family values)
    double pad[2];
};
static_assert(sizeof(SweepSums) == 128, "SweepSums layout");

// The pass schedule of one transform of 2^nh points (nh = n - 1 after the
// Hermitian halving): a first tile pass over bits [0, k1) that also forms the
// products, then column passes over [lo_i, lo_i + s_i).
struct Plan {
    int n;          // qubits
    int nh;         // transform bits = n - 1 (n >= 2)
    bool fused;     // whole transform inside one workgroup (nh <= small limit)
    int k1;         // bits of the first pass
    int npass;      // number of column passes after the first
    int ktile;      // index bits per column-pass tile (12, or 13 when that saves a pass)
    int lo[4];
    int s[4];
    int blocks_last;   // workgroups per family in the final pass
    // split-BF16 Hadamard blocks on the matrix cores for the single-workgroup transform and
    // the first pass (single precision storage; column passes stay FP32 on the VALU)
    bool mfma;
    // families per first-pass tile-sharing group asked for by a schedule (0: the default
    // policy of first_pass_group)
    int grp_req;
};

// Largest first-pass tile-sharing group (families that read one state tile once).
constexpr int GROUP_MAX = 128;

// A transform schedule: first-pass bits (12, or 15 for single precision n - 1 = 16..27),
// column-tile bits (12; 13 single precision; 15 single precision after a 15-bit first pass
// with 9..12 bits left), first-pass group (a power of two up to GROUP_MAX); 0 = the default
// choice.
struct Schedule {
    int first_bits, column_tile_bits, group;
};
// The plan of a schedule; *honoured is false (and the default plan is returned) when the
// schedule does not apply to (n, dbl).
Plan make_plan_sched(int n, bool dbl, const Schedule& sc, bool* honoured);

Plan make_plan(int n, bool dbl);
// The plan of the split-BF16 matrix-core transform: single precision, the single-workgroup
// kernel up to n - 1 = 13 bits (from n - 1 = 8; below that the FP32 kernel), else a 12-bit
// first pass and FP32 column passes.
Plan make_plan_bf16x2(int n);

// Message buffer behind pw_last_error (thread-local).
std::string& last_error_ref();

// Families per group of the first pass that share their state tiles (1, 2 or 4; more
// than 1 only for multi-pass plans of states of 16 MiB and more, and at most nb).  The
// workgroups of one tile and group run back to back on one XCD, so the tile leaves
// HBM (or the MALL) once.
int first_pass_group(const Plan& P, bool dbl, int nb);

// Grouping support for lists of families: a stable sort of nx <= SORT_MAX families by
// the top set bit of x mod 2^n (x = 0 first), xs_sorted[j] = xs[perm[j]], so that
// consecutive families share state tiles; and the per-family results of the sorted list
// put back in list order, out[perm[j]] = in[j].
constexpr int SORT_MAX = 4096;
hipError_t sort_by_top_bit(const uint64_t* xs, int n, int nx, uint64_t* xs_sorted, uint32_t* perm, hipStream_t st);
hipError_t scatter_results(const FamilyRes* in, const uint32_t* perm, int nx, FamilyRes* out, hipStream_t st);

// Optional launch timing.  For a sampled launch, take() hands out two HIP events
// that the launch attaches to the kernel's own dispatch (hipExtLaunchKernel start
// and stop events, i.e. the kernel's execution interval on its stream), and
// commit() files them.  Kernel classes: 0 fused, 1 first pass, 2 middle column
// pass, 3 final column pass, 4 reduced density matrix (mixed states).
struct LaunchTimer {
    bool (*take)(void* self, int kclass, hipEvent_t* start, hipEvent_t* stop);
    void (*commit)(void* self, int kclass, int families, hipEvent_t start, hipEvent_t stop);
    void* self;
};

// Launchers (host side, enqueue on `st`).  All return hipSuccess or the first error.
// Evaluate a batch of nb families.  If xs != nullptr the x of slot i is xs[i],
// else it is x0 + i.  Per-family results go to out[i].  max_alpha is 2 (moments
// alpha = 2 only; m[1], m[2] are NaN) or 4.  parts holds nb * blocks_last partials.
// With finalize == false a multi-pass plan stops at the partials (family i at
// parts + i * blocks_last) and out is not written: several batches can then be
// finalized by one finalize_families call.  Single-workgroup plans always write out.
// fpsi (with xs only): device array of nb state addresses, family i reads the state at
// fpsi[i] instead of psi (several states of the same n and dtype in one launch).
hipError_t eval_batch(const Plan& P, bool dbl, int max_alpha, const void* psi, const uint64_t* xs, uint64_t x0,
                      int nb, double eps, void* work, FamilyRes* parts, FamilyRes* out, hipStream_t st,
                      const LaunchTimer* tm = nullptr, bool finalize = true, const uint64_t* fpsi = nullptr);
// Per-family results of nfam families whose partials are contiguous in parts.
hipError_t finalize_families(const Plan& P, int max_alpha, const FamilyRes* parts, int64_t nfam, FamilyRes* out,
                             hipStream_t st);

// Mixed states: rho_A = Psi Psi^dagger of the first na qubits, stored family-major as
// D[x_A][a] = rho_A[a ^ x_A, a] (d_A x d_A), and the families x_A = x0 .. x0 + nb - 1 of
// the reduced state.  When make_plan(na) is not single-workgroup the families go through
// the multi-pass transform: work holds nb * 2^(na-1) points, parts nb * blocks_last.
hipError_t reduced_density(bool dbl, const void* psi, int n, int na, void* rho, hipStream_t st,
                           const LaunchTimer* tm = nullptr);
hipError_t eval_reduced_batch(bool dbl, int max_alpha, const void* rho, int na, uint64_t x0, int nb, double eps,
                              void* work, FamilyRes* parts, FamilyRes* out, hipStream_t st);

// Fixed-order sum of count per-family results.
// Partial sums of count per-family results, FAM_PER_SLOT families per slot, written to
// out[0 .. reduce_families_slots(count)) in family order.
constexpr int64_t FAM_PER_SLOT = 4096;
inline int64_t reduce_families_slots(int64_t count) { return (count + FAM_PER_SLOT - 1) / FAM_PER_SLOT; }
hipError_t reduce_families(const FamilyRes* in, int64_t count, SweepSums* out, hipStream_t st);

// Transform only (no reductions): writes the 2^nh half-spectrum G of one x into work.
hipError_t transform_one(const Plan& P, bool dbl, const void* psi, uint64_t x, void* work, hipStream_t st);
// Signed values c(x, z) from the half spectrum G (2^n doubles).
hipError_t signed_values(const Plan& P, bool dbl, const void* G, uint64_t x, double* c, hipStream_t st);

// Sum an array of batch sums (fixed order) into one.
hipError_t reduce_sweep(const SweepSums* in, int64_t count, SweepSums* out, hipStream_t st);

// State helpers.
hipError_t norm2(bool dbl, const void* psi, int n, double* d_partial, int nparts, double* d_out, unsigned* d_bad,
                 hipStream_t st);
int norm2_parts(int n);
// dst (2^n amplitudes) = src in the other precision: complex128 -> complex64 when src_dbl,
// else complex64 -> complex128.
hipError_t convert_state(bool src_dbl, const void* src, void* dst, int n, hipStream_t st);
hipError_t apply_gate2(bool dbl, void* psi, int n, int q0, int q1, const double* m16 /*host*/, hipStream_t st);
// Up to 6 two-qubit gates (local bit positions a[g], b[g] in [0, W + H), matrices
// m32[32 g ..] host) in one pass over tiles of bits [0, W) and [hb, hb + H), W + H <= 12.
hipError_t apply_gates_tile(bool dbl, void* psi, int n, int W, int hb, int H, int ng, const int* a, const int* b,
                            const double* m32, hipStream_t st);
// Two-qubit Clifford group modulo phase (host table, built once) and random brick-wall
// circuits over it: pairs q[2g], q[2g+1] and table indices idx[g].
int clifford2_count();
void clifford2_matrix(int i, double* m32);
void brickwall_clifford(int n, int n_layers, uint64_t seed, std::vector<int>& q, std::vector<int>& idx,
                        std::vector<int>* layer_start = nullptr);
hipError_t apply_diag(bool dbl, void* psi, int n, int q, const double* d2 /*host*/, hipStream_t st);

// Sampling.
// With d_off != nullptr the sample counters start at offset + *d_off (read on the
// device, so that a captured graph draws new samples on every replay).
hipError_t sample_uniform(int n, uint64_t seed, uint64_t offset, int64_t count, uint64_t* d_xs, hipStream_t st,
                          const uint64_t* d_off = nullptr);
hipError_t bump_counter(uint64_t* d_ctr, uint64_t v, hipStream_t st);
hipError_t build_cdf(bool dbl, const void* psi, int n, double* d_cdf, double* d_blk, hipStream_t st);
size_t cdf_blk_elems(int n);
hipError_t sample_marginal(int n, const double* d_cdf, uint64_t seed, uint64_t offset, int64_t count, uint64_t* d_xs,
                           hipStream_t st, const uint64_t* d_off = nullptr);

// Learned proposal (masked autoregressive network over the bits of x).
struct MadeDims {
    int n, h;
    size_t oW1, ob1, oW2, ob2, oW3, ob3, oA, total;
};
MadeDims made_dims(int n, int h);
hipError_t made_forward(const MadeDims& D, const float* P, const uint64_t* xs, const int* perm, int B, float* H1,
                        float* H2, float* O, double* logq, hipStream_t st);
hipError_t made_backward(const MadeDims& D, const float* P, const uint64_t* xs, const int* perm, const float* w,
                         float invW, int B, const float* H1, const float* H2, const float* O, float* dO, float* G1,
                         float* G2, hipStream_t st);
hipError_t made_wgrad(const MadeDims& D, const uint64_t* xs, const int* perm, int B, const float* dO, const float* G1,
                      const float* G2, const float* H1, const float* H2, float* grad, hipStream_t st);
hipError_t made_adam(float* P, const float* g, float* m, float* v, size_t count, float lr, float b1, float b2,
                     float eps, int t, hipStream_t st);
hipError_t made_sample(const MadeDims& D, const float* P, uint64_t seed, uint64_t offset, int64_t count, uint64_t* xs,
                       hipStream_t st);

}  // namespace pw
