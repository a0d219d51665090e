/*
 * pauliwht.h -- C ABI of the MI355X (gfx950) library for FWHT Pauli-string
 * evaluation: stabilizer Renyi entropies and stabilizer nullity of an N-qubit
 * state vector (Xiao & Ryu, "Exponentially Accelerated Sampling of Pauli Strings
 * for Nonstabilizerness").
 *
 * What the library computes.  For every X-bitstring x, the family
 * { <psi|P_{x,z}|psi> : z } is the Walsh-Hadamard transform over b of
 *     f_x(b) = conj(psi(b)) psi(b ^ x)                       (Pauli labelling section)
 * and one fast transform gives all 2^N values at O(N) cost per string.  Fused
 * reductions over z give, per family,
 *     p(x)   = m_{1;x} = sum_z |F|^2 / d                     (exact x-marginal)
 *     ent(x) = sum_z |F|^2 log2 |F|^2                         (Shannon term, alpha = 1)
 *     m[a]   = m_{a+2;x} = sum_z |F|^{2(a+2)} / d^{a+2}      (partial moments, alpha = 2, 3, 4)
 *     nu(x)  = #{ z : ||F| - 1| < eps }                       (nullity count)
 * and the estimators combine them (Algorithm 1 for the exact sweep; the Monte
 * Carlo section and its error formula, Eq. stdM, for sampling).
 *
 * Conventions.
 *   - Qubit j is bit j of the basis index (little endian); x and z are bit masks.
 *   - The Hermitian Pauli of label (x, z) is i^{|x&z|} X^x Z^z (Y = iXZ), so
 *     <psi|P|psi> = (-i)^{|x&z|} F_x(z), which is real.
 *   - States are contiguous, interleaved (re, im): PW_C128 = 2 doubles per
 *     amplitude (the transform runs in FP64), PW_C64 = 2 floats (FP32 transform).
 *     Per-family sums are accumulated in FP64 in a fixed order, so results are
 *     bitwise reproducible run to run.
 *   - M_alpha = log2(S_alpha)/(1 - alpha) - N (Eq. SRE-def), M_1 = -(1/d) sum_x ent(x)
 *     (the alpha -> 1 limit), nu = N - log2(nu_cnt).
 *
 * Ownership.  Device buffers (the state, the workspace) belong to the caller and
 * are borrowed; the library never frees them.  Host arrays passed in or out are
 * caller-allocated.  The library allocates device memory of its own for the
 * workspace when none was set, for pw_mixed's reduced density matrix and pass
 * buffers, and for the learned proposal (pw_made_init); it owns these, reuses
 * them while large enough, and frees them at pw_ctx_destroy.
 *
 * Streams.  All device work of a context is enqueued on the stream given at
 * creation (NULL = the default stream).  Calls that return host results
 * synchronise that stream before returning.
 *
 * Errors.  Every call returns a pw_status.  Out-parameters are written only on
 * PW_OK.  pw_last_error() gives a message for the last failing call of the
 * calling thread.  A context must not be used from two threads at once.
 */
#ifndef PAULIWHT_H
#define PAULIWHT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#if defined(__GNUC__) || defined(__clang__)
#define PW_API __attribute__((visibility("default")))
#else
#define PW_API
#endif

typedef struct pw_ctx_s* pw_ctx;

typedef enum {
    PW_OK = 0,
    PW_ERR_ARG = 1,             /* null pointer, bad enum, bad count              */
    PW_ERR_RANGE = 2,           /* qubit count or x outside the supported range   */
    PW_ERR_NOT_NORMALIZED = 3,  /* |<psi|psi> - 1| above tolerance, or NaN/Inf     */
    PW_ERR_NO_STATE = 4,        /* no state bound to the context                   */
    PW_ERR_WORKSPACE = 5,       /* workspace too small                             */
    PW_ERR_HIP = 6,             /* a HIP runtime call failed                       */
    PW_ERR_TOLERANCE = 7,       /* nullity count is not a power of two            */
    PW_ERR_UNSUPPORTED = 8      /* valid request the library does not handle       */
} pw_status;

typedef enum { PW_C128 = 0, PW_C64 = 1 } pw_dtype;

/* Arithmetic of the product and the transform (pw_set_precision).  The reductions over z,
 * the logarithms and the nullity test always accumulate in FP64. */
typedef enum {
    PW_PREC_AUTO = 0,    /* follows the storage: FP64 for complex128, FP32 for complex64       */
    PW_PREC_F64 = 1,     /* FP64 (a complex64 state is widened into a library-owned copy)       */
    PW_PREC_F32 = 2,     /* FP32 (a complex128 state is rounded into a library-owned copy)      */
    PW_PREC_BF16X2 = 3   /* split-BF16 Hadamard blocks on the matrix cores, FP32 accumulate     */
} pw_prec;

typedef enum {
    PW_SAMPLER_UNIFORM_NZ = 0,  /* x uniform over F_2^N \ {0} (Monte Carlo section)  */
    PW_SAMPLER_MARGINAL_NZ = 1  /* x ~ p(x | x != 0), p the exact x-marginal          */
} pw_sampler;

/* Per-family results (one per x). */
typedef struct {
    uint64_t x;
    double p;          /* m_{1;x}: exact x-marginal                                  */
    double ent;        /* sum_z |F|^2 log2 |F|^2                                      */
    double m[3];       /* m_{alpha;x}, alpha = 2, 3, 4                                */
    double gap;        /* max |F| below 1 - eps (-1 if none): margin of the nullity test */
    uint64_t nu;       /* #{z : ||F| - 1| < eps}                                      */
} pw_xres;

/* Whole-state results of pw_exact / pw_mc. */
typedef struct {
    double S[3];       /* sum_x m_{alpha;x}, alpha = 2, 3, 4 (estimate for pw_mc)     */
    double S_se[3];    /* standard error of S (0 for pw_exact)                        */
    double M[3];       /* M_alpha                                                      */
    double M_se[3];    /* sigma_S / (|1-alpha| ln2 S)  (Eq. stdM)                      */
    double L, L_se;    /* sum_x ent(x) and its standard error                          */
    double M1, M1_se;  /* M_1 = -L/d                                                   */
    double P;          /* sum_x p(x) over the families evaluated (1 for pw_exact)     */
    double nullity;    /* N - log2 nu_cnt (pw_exact only; NaN for pw_mc)               */
    uint64_t nu_cnt;   /* sum_x nu(x) (pw_exact only)                                  */
    uint64_t n_samples;/* families evaluated, x = 0 included                           */
    double r[3];       /* pw_mc: sample sd of the per-draw terms / their mean;          *
                        * pw_exact: r_alpha = Std_{x!=0}(m_{alpha;x}) / E_x[m_{alpha;x}]  *
                        * (Supplemental, brick-wall circuits: the spread that sets the    *
                        * Monte Carlo sample count)                                       */
    double gap;        /* max over families of gap                                     */
} pw_result;

/* Message for the last failing call on this thread ("" if none).  Valid until
 * the next pw_* call on this thread. */
PW_API const char* pw_last_error(void);

/* Library version string. */
PW_API const char* pw_version(void);

/* Create a context on HIP device `device`, enqueuing on `hip_stream`
 * (a hipStream_t, borrowed; NULL = default stream). */
PW_API pw_status pw_ctx_create(pw_ctx* out, int device, void* hip_stream);
PW_API pw_status pw_ctx_destroy(pw_ctx ctx);

/* Device bytes of workspace needed to evaluate up to `x_batch` families of an
 * n-qubit state of the given dtype per launch, including the two FP64 prefix
 * tables of the marginal sampler (2 * 2^n doubles).  1 <= n <= 32. */
PW_API pw_status pw_workspace_size(int n_qubits, pw_dtype dtype, int x_batch, size_t* bytes);

/* Lend a device buffer (256-byte aligned) as workspace; the library carves all
 * its scratch from it.  Pass NULL/0 to return to library-owned scratch.  A lent
 * buffer runs the largest launch it holds.  Library-owned scratch is sized for
 * the default launch: up to 256 MiB of half spectra (at most 256 families), and
 * up to sixteen families (64 once a family's half spectrum is 64 MiB or more; within
 * 16 GiB) for states of 16 MiB and more, whose
 * first pass runs them in one group sharing the state's tiles; lists are
 * then evaluated in order of the top bit of x and the results put back in list
 * order. */
PW_API pw_status pw_set_workspace(pw_ctx ctx, void* dev_ptr, size_t bytes);

/* Bind a device state (2^n amplitudes, borrowed, 256-byte aligned).  Computes
 * <psi|psi> in FP64 (one streaming read) and rejects NaN/Inf or a norm off by
 * more than 1e-10 (PW_C128) / 1e-5 (PW_C64): the method assumes a normalised
 * state (Pauli expansion paragraph).  norm2_out may be NULL. */
PW_API pw_status pw_state_bind(pw_ctx ctx, int n_qubits, pw_dtype dtype, void* dev_psi, double* norm2_out);

/* Copy a host state into the caller's device buffer dev_dst, then bind it. */
PW_API pw_status pw_state_upload(pw_ctx ctx, int n_qubits, pw_dtype dtype, const void* host_psi,
                          void* dev_dst, double* norm2_out);

/* Apply a gate list to the bound state, in place, in order (Clifford
 * preconditioning section: a random brick-wall Clifford circuit applied before
 * sampling; also used to prepare T-doped circuit states).
 *   kinds[g] = 2: dense 4x4 unitary on qubits (qubits[2g], qubits[2g+1]), acting on
 *                 the local index b_{q0} + 2 b_{q1};
 *   kinds[g] = 1: diagonal gate diag(d0, d1) on qubit qubits[2g].
 *   mats: 16 complex doubles (interleaved) per gate, row-major; a diagonal gate
 *         keeps (d0, d1) in its first two entries.
 * Host arrays, copied before the call returns.  The state is not re-normalised. */
PW_API pw_status pw_apply_gates(pw_ctx ctx, int n_gates, const int* kinds, const int* qubits, const double* mats);

/* Clifford preconditioning (Clifford preconditioning section): n_layers brick-wall
 * layers of two-qubit Cliffords, each drawn uniformly from the 11520-element
 * two-qubit Clifford group modulo phase, applied in place to the bound state.  Layer
 * l acts on the pairs (i, i+1) for i = l mod 2, l mod 2 + 2, ...; periodic for even n
 * (odd layers include (n-1, 0), every layer has n/2 gates), open for odd n.  Gate g
 * takes the group element floor(W 11520 / 2^64), W the first 64-bit word of
 * Philox4x32-10 with counter (g, 0, "CLIF") and key seed.  M_alpha and the nullity
 * are unchanged; the exact marginal changes (the paper uses n_layers = 2n).
 * Errors: PW_ERR_NO_STATE, PW_ERR_RANGE (n < 2), PW_ERR_ARG (n_layers < 0). */
PW_API pw_status pw_precondition(pw_ctx ctx, int n_layers, uint64_t seed);

/* The gate list pw_precondition applies for (n, n_layers, seed): *n_gates gates,
 * pairs qubits[2g], qubits[2g+1] and 4x4 matrices mats[32g ..] (interleaved complex,
 * row-major, local index b_{q0} + 2 b_{q1}).  Host arrays of the caller; null arrays
 * are skipped (call once with nulls for the count).  No GPU needed. */
PW_API pw_status pw_precondition_circuit(int n, int n_layers, uint64_t seed, int64_t* n_gates, int* qubits,
                                         double* mats);

/* The two-qubit Clifford group modulo phase as the library enumerates it (breadth-first
 * from the identity over H, S on either qubit and CNOT either way; each element scaled
 * so that its first nonzero entry is real positive): *count = 11520 matrices into
 * mats[32 i ..] when mats is not null.  No GPU needed. */
PW_API pw_status pw_clifford2_table(int* count, double* mats);

/* Evaluate the families of the host list xs[0..n_x) (any x < 2^n, repeats
 * allowed) and write one pw_xres per x to the host array out.  eps is the
 * nullity tolerance (the paper suggests 1e-7 in FP64; use >= 1e-4 with PW_C64). */
PW_API pw_status pw_eval_x(pw_ctx ctx, const uint64_t* xs, int64_t n_x, double eps, pw_xres* out);

/* Same, with device arrays, enqueued without synchronising (graph-capturable
 * when a workspace is set).  The list is not checked on the host: each x is
 * taken modulo 2^n (bits at or above n are ignored, and the result records the
 * reduced x), so no list makes the kernels read outside the state. */
PW_API pw_status pw_eval_x_device(pw_ctx ctx, const uint64_t* d_xs, int64_t n_x, double eps, pw_xres* d_out);

/* The signed expectation values c(x, z) = (-i)^{|x&z|} F_x(z) of one family,
 * z = 0..2^n-1, into the host array c (2^n doubles).  1 <= n <= 26. */
PW_API pw_status pw_family_values(pw_ctx ctx, uint64_t x, double* c);

/* Draw n x-strings on the device (Philox4x32-10 counters keyed by seed; sample i
 * uses counter offset + i) into the host array xs_out.  Marginal sampling draws
 * x = b1 ^ b2 with b1, b2 ~ |psi|^2 by inverse CDF and redraws x = 0 (at most
 * 64 attempts; a sample still 0 then takes the pair directly from its law given
 * b1 != b2: b1 ~ q (T - q), b2 ~ q without b1).  The draws follow
 * p(x) / (1 - p(0)) on x != 0 exactly for any p(0) < 1; x = 0 is returned only
 * when |psi|^2 is a point mass. */
PW_API pw_status pw_sample_x(pw_ctx ctx, pw_sampler sampler, uint64_t seed, uint64_t offset, int64_t n,
                      uint64_t* xs_out);

/* Exact enumeration of all 4^n Pauli strings (Algorithm 1): every x is
 * evaluated; S_alpha, M_alpha, M_1, nu_cnt and the nullity are returned.
 * Returns PW_ERR_TOLERANCE (with the result still written) when nu_cnt is not a
 * power of two.  n <= 26. */
PW_API pw_status pw_exact(pw_ctx ctx, double eps, pw_result* out);

/* Monte Carlo estimate (Monte Carlo section).  x = 0 is always evaluated and
 * counted; further x are drawn `batch` at a time from `sampler` and evaluated,
 * until the standard error of M_2 is <= target_se (after at least 2 batches) or
 * max_samples families have been evaluated.  The uniform sampler uses the
 * paper's estimator S = m_0 + (d-1) mean(m_x); the marginal sampler uses
 * S = m_0 + (1 - p(0)) mean(m_x / p(x)). */
PW_API pw_status pw_mc(pw_ctx ctx, pw_sampler sampler, double eps, int batch, uint64_t max_samples,
                double target_se, uint64_t seed, pw_result* out);

/* Monte Carlo with the sampler chosen from a pilot.  The number of families a target
 * error needs grows as the square of the relative spread r_2 = sd(y)/S of the per-draw
 * terms (Monte Carlo section, Eq. stdM), and which sampler spreads less depends on the
 * state.  A pilot of `pilot` exact-marginal draws (Philox key seed ^ 0x50494C4F54; not
 * counted in the result) estimates both spreads: the marginal's from its own terms
 * (1 - p0) m_x / p(x), the uniform sampler's from the same draws reweighted to the uniform
 * law (second moment sum_{x != 0} (d - 1) m_x^2 = E[(d - 1)(1 - p0) m_x^2 / p(x)]).  Since
 * m_x <= p(x)/d, the families with large m_x that dominate the uniform sampler's variance
 * are those the marginal draws most often, which a short uniform pilot tends to miss.
 * The sampler with the smaller estimate runs pw_mc(ctx, chosen, eps, batch, max_samples,
 * target_se, seed) -- bitwise that call's result.  A state whose marginal has no mass on
 * x != 0 takes the uniform sampler.  Optional outputs: *chosen, pilot_r2[2] (uniform,
 * marginal; NaN when the marginal pilot could not run). */
PW_API pw_status pw_mc_auto(pw_ctx ctx, double eps, int batch, uint64_t max_samples, double target_se,
                            uint64_t seed, int64_t pilot, pw_sampler* chosen, double* pilot_r2, pw_result* out);

/* ---------------------------------------------------------------------------
 * Learned proposal over X-bitstrings (not in the paper; an importance-sampling
 * proposal for the Monte Carlo estimator).  A masked autoregressive network
 * (MADE, Germain et al. 2015) n -> hidden -> hidden -> n with ReLU hidden layers,
 * Bernoulli outputs and direct input->output links, FP32 on the device.  Bit i of
 * x is input i; hidden unit k has degree (k mod (n-1)) + 1, so output i depends on
 * bits j < i.  Parameters are a flat array (host side: doubles) in the layout
 *   W1T[n*hidden] (i*hidden + k), b1[hidden], W2T[hidden*hidden] (kk*hidden + k),
 *   b2[hidden], W3T[hidden*n] (kk*n + i), b3[n], AT[n*n] (j*n + i, used for j < i).
 * The network lives in the context (library-owned device memory, freed at
 * pw_ctx_destroy).  2 <= n <= 32, hidden in {64, 128, 256}.
 * --------------------------------------------------------------------------- */
PW_API pw_status pw_made_param_count(int n, int hidden, size_t* count);
/* (Re)create the network with the given initial parameters (host array, copied) and
 * reset the Adam state. */
PW_API pw_status pw_made_init(pw_ctx ctx, int n, int hidden, const double* params);
PW_API pw_status pw_made_get(pw_ctx ctx, double* params);
/* log q(x) for the host list xs (host output, FP64 from FP32 logits). */
PW_API pw_status pw_made_logq(pw_ctx ctx, const uint64_t* xs, int64_t count, double* logq);
/* Loss -(sum_b w_b log q(x_b)) / sum_b w_b and its gradient (one batch, count <= 4096). */
PW_API pw_status pw_made_grad(pw_ctx ctx, const uint64_t* xs, const double* w, int64_t count, double* loss,
                              double* grad);
/* Weighted maximum likelihood with Adam (beta1 0.9, beta2 0.999, eps 1e-8): `epochs`
 * passes over the samples in minibatches, shuffled per epoch from `seed`.  Optional
 * final_loss is the full-set loss after training. */
PW_API pw_status pw_made_train(pw_ctx ctx, const uint64_t* xs, const double* w, int64_t count, int epochs,
                               int minibatch, double lr, uint64_t seed, double* final_loss);
/* Draws from q(x | x != 0): bit j of sample i compares u = (W0 >> 40) 2^-24 from
 * Philox(ctr = (offset+i, attempt*64 + j, "MADE"), key = seed) with the logistic of
 * output j (redraw when x = 0, at most 64 attempts; 0 is returned if all fail). */
PW_API pw_status pw_made_sample(pw_ctx ctx, uint64_t seed, uint64_t offset, int64_t count, uint64_t* xs_out);
/* Monte Carlo with the learned proposal: x = 0 evaluated; `pilot` draws from the exact
 * marginal are evaluated and the network is trained on them with weights m_{2;x}/p(x)
 * (targets the zero-variance proposal t(x) ~ m_{2;x}); the same pilot estimates the spread
 * of the two plain samplers (as in pw_mc_auto) and the one that spreads less becomes the
 * defensive component q_def (uniform over x != 0, or the exact marginal p(.|x!=0)); then
 * draws from the mixture q = lambda q_def + (1-lambda) q_theta(.|x!=0) (per-sample choice
 * from Philox stream "MIXC") are weighted exactly by m_{alpha;x}/q(x), until the standard
 * error of M_2 is <= target_se or max_samples families (x = 0 included; pilot families not
 * counted). */
PW_API pw_status pw_mc_learned(pw_ctx ctx, double eps, int batch, uint64_t max_samples, double target_se,
                               uint64_t seed, double lambda, int64_t pilot, int epochs, int minibatch, double lr,
                               pw_result* out);

/* pw_mc_learned with plain sampling kept as the judge: the network trains on the first
 * three quarters of the pilot, and on the held-out quarter the second moment of m/g is
 * estimated for g = uniform, exact marginal and the mixture (E_{p_c}[m^2 / (g p_c)], p_c the
 * marginal on x != 0).  If a plain sampler is predicted to spread less than the mixture,
 * that sampler runs (pw_mc on the stream seed + 0x9E3779B97F4A7C15) instead.  *chosen: 0
 * uniform, 1 marginal, 2 mixture with the uniform, 3 mixture with the marginal;
 * predicted_r2[3]: the held-out r_2 of uniform, marginal and mixture.  pilot >= 8. */
PW_API pw_status pw_mc_learned_auto(pw_ctx ctx, double eps, int batch, uint64_t max_samples, double target_se,
                                    uint64_t seed, double lambda, int64_t pilot, int epochs, int minibatch,
                                    double lr, int* chosen, double* predicted_r2, pw_result* out);

/* Stabilizer Renyi entropy of the reduced state rho_A on the first n_a qubits
 * (Supplemental Material, mixed states, Eq. Msre-mixed):
 *   M_alpha(rho_A) = log2(W_alpha)/(1 - alpha) - n_a - S_2(rho_A),
 *   W_alpha = sum_{P on A} |Tr(rho_A P)|^{2 alpha} / d_A^alpha,  S_2 = -log2 Tr rho_A^2.
 * rho_A = Psi Psi^dagger (Psi[a, e] = psi(a + 2^{n_a} e)) is formed on the device
 * (the tiles on and above the diagonal, on the matrix cores; it is Hermitian) and
 * stored family by family, then every x_A family is the n_a-bit WHT of
 * h(a) = rho_A[a ^ x_A, a] (one workgroup per family up to n_a = 14 (c64) / 13
 * (c128), the multi-pass transform above).  1 <= n_a <= min(n, 16); rho_A (d_A^2
 * amplitudes: 32 GiB for c64, 64 GiB for c128 at n_a = 16) and the pass buffers
 * are library-owned. */
typedef struct {
    double W[3];        /* W_alpha, alpha = 2, 3, 4 (NaN above pw_set_moments)     */
    double purity;      /* Tr rho_A^2 = sum_{P on A} |c_P|^2 / d_A                 */
    double S2;          /* -log2 purity                                              */
    double M[3];        /* M_alpha(rho_A)                                            */
    double L;           /* sum_{P on A} c_P^2 log2 c_P^2                             */
    uint64_t families;  /* 2^{n_a}                                                   */
} pw_mixed_result;
PW_API pw_status pw_mixed(pw_ctx ctx, int n_a, double eps, pw_mixed_result* out);

/* Autotuning of the transform schedule of the bound state, timed on a list of uniformly
 * drawn x (4 x the workspace batch, at most 4096; the sorted, grouped path that Monte Carlo
 * steps and device lists take).  Stage 1, at the workspace's launch size: every plan
 * variant that applies -- first pass over the low 12 index bits, or (single precision,
 * n - 1 = 16..27) over 15 bits; column tiles of 12 or 13 bits (single precision), or of
 * 15 bits after a 15-bit first pass -- crossed with first-pass tile-sharing groups of 1, 2,
 * 4, ..., 128 families (up to the launch size).  Stage 2, for the fastest: up to 6 launch sizes (the workspace batch
 * and its halvings, none below the group).  The result is recorded per (device, n,
 * arithmetic) for every context of the process (pw_autotune_save / pw_autotune_load keep
 * it across processes) and takes effect on this context unless pw_set_schedule fixed one.
 * Results do not depend on the launch size or the group; the plan variant changes the
 * order of the FP32 roundings only.  Optional outputs (stage 2): candidates[i],
 * us_per_family[i] (arrays of >= 6), n_candidates. */
PW_API pw_status pw_autotune(pw_ctx ctx, int* best_batch, int* candidates, double* us_per_family, int* n_candidates);

/* Fix the schedule of this context (0 = the tuned or default choice for that part):
 * first_bits 12 or 15, column_tile_bits 12, 13 or 15, group 1, 2, 4, ..., 128 families per
 * first-pass tile-sharing group, batch families per launch (at most the workspace's).
 * PW_ERR_UNSUPPORTED when the schedule does not apply to the bound state; a later bind of a
 * state it does not apply to takes the default plan. */
PW_API pw_status pw_set_schedule(pw_ctx ctx, int first_bits, int column_tile_bits, int group, int batch);
/* The schedule in effect for the bound state (0 for the single-workgroup plans). */
PW_API pw_status pw_get_schedule(pw_ctx ctx, int* first_bits, int* column_tile_bits, int* group, int* batch);
/* Write every tuned schedule of the process to a text file (one line per device
 * architecture, n and arithmetic), or read such a file and take its entries for the
 * visible devices of the same architecture (*loaded = entries taken). */
PW_API pw_status pw_autotune_save(const char* path);
PW_API pw_status pw_autotune_load(const char* path, int* loaded);

/* Several states of different sizes in one call: family xs[i] of state
 * states[state_idx[i]], results to out[i] (host arrays).  One workspace serves all
 * states, sized for the largest layout.  States of the same n and dtype form a class whose
 * families run as one list, launches spanning its states (each family reads its own
 * state's address), at that size's families per launch; results are bitwise those of one
 * pw_eval_x call per state.  Every state with families is norm-checked before any family is
 * evaluated (PW_ERR_NOT_NORMALIZED names the first bad one; out is then untouched).
 * The call synchronises the stream twice, staging x lists and results through
 * library-owned pinned host memory.  The bound state of the context is kept, also
 * when the call fails, except when its workspace, freed to grow for a larger state,
 * cannot be allocated again: then no state is bound (PW_ERR_NO_STATE until the next
 * bind or upload). */
typedef struct {
    void* psi;         /* device amplitudes, 256-byte aligned, borrowed */
    int n;
    pw_dtype dtype;
} pw_state_ref;
PW_API pw_status pw_eval_states(pw_ctx ctx, int nstates, const pw_state_ref* states, const int* state_idx,
                                const uint64_t* xs, int64_t n_x, double eps, pw_xres* out);

/* Arithmetic of every later family evaluation of this context (pw_eval_x, pw_eval_x_device,
 * pw_exact, pw_mc, pw_mc_auto, pw_mc_learned, pw_autotune); pw_family_values, pw_mixed and
 * the samplers keep the storage precision, and pw_eval_states evaluates every state in its
 * storage precision except that complex64 states follow PW_PREC_BF16X2.  A state stored in the other
 * precision is converted into a library-owned device copy (2^n amplitudes) before the next
 * evaluation and again after pw_apply_gates / pw_precondition; the workspace is planned for
 * the compute precision (size a lent workspace with pw_workspace_size of that dtype).
 * PW_PREC_BF16X2 (Eq. for the FWHT written as Hadamard blocks, H_16 = H^{(x)4}): the product
 * is formed in FP32, and the low 8 index bits of every tile of the transform go through two
 * 16 x 16 Hadamard steps on the matrix cores (v_mfma_f32_16x16x32_bf16) with each FP32 input
 * split into two BF16 parts x = hi + lo (residual |x - hi - lo| <= 2^-18 |x|) and FP32
 * accumulation; the other bits run as FP32 butterflies.  Error bound per value:
 * |dF| <= (2 * 2^-18 + (n + 12) * 2^-24) * sum_b |f_x(b)| (<= that factor, Cauchy-Schwarz).
 * The single-workgroup kernel (n - 1 <= 13) takes this path from n = 9; below that the FP32
 * kernel runs.  Use a nullity tolerance of at least 1e-4 with PW_PREC_F32 or BF16X2; a
 * nullity count that is not a power of two still returns PW_ERR_TOLERANCE from pw_exact. */
PW_API pw_status pw_set_precision(pw_ctx ctx, pw_prec prec);

/* Progress of long Monte Carlo estimates (pw_mc, pw_mc_auto and the plain fallback of
 * pw_mc_learned_auto): after a sampling step, at most once per every_seconds of wall time,
 * fn(user, families evaluated so far (x = 0 included), current M_2, its standard error) is
 * called on the calling thread.  fn = NULL switches it off (the default). */
typedef void (*pw_progress_fn)(void* user, uint64_t families, double M2, double M2_se);
PW_API pw_status pw_set_progress(pw_ctx ctx, pw_progress_fn fn, void* user, double every_seconds);

/* Test support for the error paths: every later HIP call of one class made by this
 * context fails before it is issued (fault_class 1 = device or pinned allocation, 2 =
 * kernel launch, 3 = copy; 0 = none, the default), so that a test can check that the
 * failing call returns PW_ERR_HIP and leaves the context usable.  No GPU work is
 * involved; the setting stays until changed. */
PW_API pw_status pw_inject_fault(pw_ctx ctx, int fault_class);

/* Graph replay for pw_mc (off by default): when enabled, one sampling step
 * (device-side draws whose counters come from a device counter, evaluation of their
 * families in launches of the workspace batch, counter increment) is captured once
 * per pw_mc call as a HIP graph on a private non-blocking stream and replayed for
 * every full step; steps of up to 4096 draws.  Results are bitwise those of the
 * eager path.  Launches inside replays are not seen by pw_timing_*. */
PW_API pw_status pw_set_graphs(pw_ctx ctx, int enable);

/* Highest moment order computed per family: 4 (default: alpha = 2, 3, 4) or 2
 * (alpha = 2 only; m[1], m[2], S[1], S[2], M[1], M[2] are then NaN).  M_1, p(x)
 * and the nullity count are always computed. */
PW_API pw_status pw_set_moments(pw_ctx ctx, int max_alpha);

/* Measurement support.  pw_timing_enable(ctx, k) attaches a pair of HIP events to
 * the dispatch of every k-th launch of each kernel class (k = 0 disables; the
 * events bracket the kernel's execution on the context stream): class 0 =
 * single-workgroup family kernel (small n), 1 = first transform pass (products and
 * the low 12 index bits, 15 for single precision n = 23..28), 2 = middle column
 * pass, 3 = final column pass with the reductions, 4 = the reduced density matrix of
 * pw_mixed (families: 1 per launch).  pw_timing_read synchronises the
 * recorded events and returns, for one class, the number of timed launches,
 * their summed duration in milliseconds and the families they processed.
 * pw_timing_reset clears the accumulators. */
PW_API pw_status pw_timing_enable(pw_ctx ctx, int every);
PW_API pw_status pw_timing_read(pw_ctx ctx, int kclass, uint64_t* samples, double* total_ms, uint64_t* families);
PW_API pw_status pw_timing_reset(pw_ctx ctx);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): pw_eval_x_device without a context or
 * a workspace.  The families of the device list d_xs[0..n_x) (each x taken modulo 2^n)
 * of the device state dev_psi (2^n amplitudes of dtype, 256-byte aligned, borrowed,
 * not norm-checked) are written to the device array d_out in list order, moments up to
 * alpha = 4; the work is enqueued on hip_stream (a hipStream_t of the calling thread's
 * current device; NULL = default stream) without synchronising.  The kernels are those of
 * pw_eval_x_device, with results bitwise equal to it.  Their scratch is a static device
 * array of 128 MiB per GPU (held until the process ends): complex64 states up to n = 24,
 * complex128 up to n = 23; larger states return PW_ERR_WORKSPACE.  No device or host
 * memory is allocated.  Calls that overlap on one GPU share that scratch and race:
 * serialise them (one stream, or events).  Errors as elsewhere (pw_last_error). */
PW_API pw_status pw_eval_x_noalloc(void* hip_stream, int n_qubits, pw_dtype dtype, const void* dev_psi,
                                   const uint64_t* d_xs, int64_t n_x, double eps, pw_xres* d_out);

#ifdef __cplusplus
}
#endif
#endif
