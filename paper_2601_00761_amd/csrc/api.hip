// C ABI of libpauliwht (declared in include/pauliwht.h): contexts, workspace
// carving, state binding, gate lists, per-family evaluation, exact enumeration
// (Algorithm 1) and the Monte Carlo estimators (Monte Carlo section, Eq. stdM).
#include "common.h"
#include "pauliwht.h"
#include "philox.h"

#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <algorithm>
#include <chrono>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

using namespace pw;

namespace {

thread_local std::string g_err;

}  // namespace

// The calling thread's message buffer, shared with the entry point of noalloc.hip.
std::string& pw::last_error_ref() { return g_err; }

namespace {

pw_status fail(pw_status s, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
pw_status fail(pw_status s, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return s;
}

#define PW_HIP(call)                                                                          \
    do {                                                                                      \
        hipError_t e_ = (call);                                                               \
        if (e_ != hipSuccess) return fail(PW_ERR_HIP, "%s: %s", #call, hipGetErrorString(e_)); \
    } while (0)

constexpr int MAX_QUBITS = 32;
constexpr int PW_KCLASSES = 5;   // timed kernel classes (see pw_timing_enable)
constexpr int EXACT_MAX_QUBITS = 26;
constexpr int FAMILY_VALUES_MAX_QUBITS = 26;
constexpr int MIXED_MAX_QUBITS = 16;   // n_a: rho_A takes 4^16 amplitudes (32 / 64 GiB)
constexpr int SWEEP_SLOTS = 16384;   // partial sums of an exact sweep (4096 families each)
constexpr int64_t EXACT_CHUNK = 1 << 20;  // families per chunk of an exact sweep
constexpr int MAX_BATCH = 4096;

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

size_t esize(pw_dtype dt) { return dt == PW_C128 ? 16 : 8; }

// Workspace layout for (n, dtype, batch).
struct Layout {
    size_t work, parts, xs, xres, xsort, perm, xres2, fam, sweep, cdf, cdfblk, norm, ctr, total;
    int64_t parts_fams;  // families whose final-pass partials the parts region holds
    int64_t xcap;        // x values / per-family results the staging regions hold
};

// Partials of several batches are kept (up to 16 batches, 16 MiB) so that one
// finalize launch serves them all.
constexpr size_t PARTS_BYTES_MAX = (size_t)16 << 20;
constexpr int PARTS_GROUP_MAX = 16;

Layout layout_for(int n, pw_dtype dt, int batch) {
    const bool dbl = dt == PW_C128;
    const Plan P = make_plan(n, dbl);
    Layout L{};
    const size_t half = (size_t)1 << (n - 1);
    size_t work = P.fused ? 0 : (size_t)batch * half * esize(dt);
    if (n <= FAMILY_VALUES_MAX_QUBITS) {
        const size_t fam = align256(half * esize(dt)) + ((size_t)1 << n) * sizeof(double);
        if (fam > work) work = fam;
    }
    size_t off = 0;
    L.work = off;
    off += align256(work);
    L.parts = off;
    // final-pass partials: as many as the smallest column tile (2^12 points) of any schedule
    const size_t blocks = P.fused ? 1 : ((size_t)1 << (P.nh - 12));
    const size_t per_batch = (size_t)batch * blocks * sizeof(FamilyRes);
    size_t group = P.fused ? 1 : PARTS_BYTES_MAX / per_batch;
    if (group < 1) group = 1;
    if (group > (size_t)PARTS_GROUP_MAX) group = PARTS_GROUP_MAX;
    L.parts_fams = (int64_t)group * batch;
    off += align256(group * per_batch);
    // x lists and per-family results are staged MAX_BATCH at a time whatever the batch, so
    // that host lists cross the bus in few copies and Monte Carlo steps hold a whole batch
    L.xcap = MAX_BATCH;
    L.xs = off;
    off += align256((size_t)L.xcap * sizeof(uint64_t));
    L.xres = off;
    off += align256((size_t)L.xcap * sizeof(FamilyRes));
    // a list sorted by top bit for tile-sharing groups, its order and its results
    static_assert(MAX_BATCH <= SORT_MAX, "sorted lists are staged MAX_BATCH at a time");
    L.xsort = off;
    off += align256((size_t)L.xcap * sizeof(uint64_t));
    L.perm = off;
    off += align256((size_t)L.xcap * sizeof(uint32_t));
    L.xres2 = off;
    off += align256((size_t)L.xcap * sizeof(FamilyRes));
    L.fam = off;
    const int64_t chunk = ((int64_t)1 << n) < EXACT_CHUNK ? ((int64_t)1 << n) : EXACT_CHUNK;
    off += align256((size_t)chunk * sizeof(FamilyRes));
    L.sweep = off;
    off += align256((size_t)(SWEEP_SLOTS + 1) * sizeof(SweepSums));
    L.cdf = off;   // marginal-sampler tables: prefix sums of q, then of q (T - q)
    off += align256(((size_t)2 << n) * sizeof(double));
    L.cdfblk = off;
    off += align256(2 * cdf_blk_elems(n) * sizeof(double));
    L.norm = off;
    off += align256((size_t)(norm2_parts(n) + 2) * sizeof(double));
    L.ctr = off;
    off += 256;
    L.total = off;
    return L;
}

int default_batch(int n, pw_dtype dt) {
    const Plan P = make_plan(n, dt == PW_C128);
    if (P.fused) return MAX_BATCH;
    const size_t per = ((size_t)1 << (n - 1)) * esize(dt);
    size_t b = ((size_t)256 << 20) / per;
    if (b < 1) b = 1;
    if (b > 256) b = 256;
    // power of two
    size_t p = 1;
    while (p * 2 <= b) p *= 2;
    // states of 16 MiB and more: launches of up to sixteen families, which the first pass
    // runs in one tile-sharing group (up to 16 GiB of half spectra); up to 64 once a family's
    // half spectrum is 64 MiB or more, where the MALL holds no batch anyway (measured per
    // family against launches of 16: complex64 N = 24 -4 %, 26 -3.5 %, 27 -3 %, complex128
    // N = 24 -2 %)
    const size_t cap = per >= ((size_t)64 << 20) ? 64 : 16;
    while (p < cap && first_pass_group(P, dt == PW_C128, 16) > 1 && 2 * p * per <= ((size_t)16 << 30)) p *= 2;
    return (int)p;
}

}  // namespace

struct pw_ctx_s {
    int device = 0;
    hipStream_t stream = nullptr;
    // workspace
    char* ws = nullptr;
    size_t ws_bytes = 0;
    bool ws_owned = false;
    // bound state
    void* psi = nullptr;
    int n = 0;
    pw_dtype dtype = PW_C128;
    bool bound = false;
    int batch = 1;       // families per launch the workspace is carved for
    int run_batch = 1;   // families per launch actually used (<= batch; autotuned)
    Layout L{};
    Plan P{};
    bool cdf_valid = false;
    int max_alpha = 4;
    // launch timing (measurement)
    int timing_every = 0;
    uint64_t launches[PW_KCLASSES] = {};
    struct Pair {
        hipEvent_t a, b;
        int kclass, families;
    };
    std::vector<Pair> pending;
    std::vector<hipEvent_t> pool;
    double total_ms[PW_KCLASSES] = {};
    uint64_t samples[PW_KCLASSES] = {};
    uint64_t sampled_families[PW_KCLASSES] = {};
    LaunchTimer timer{};
    // learned proposal (library-owned device buffers)
    struct Made {
        bool ready = false;
        MadeDims D{};
        int t = 0;
        int maxB = 0;
        void* block = nullptr;
        float *P = nullptr, *g = nullptr, *m = nullptr, *v = nullptr;
        float *H1 = nullptr, *H2 = nullptr, *O = nullptr, *dO = nullptr, *G1 = nullptr, *G2 = nullptr;
        double* logq = nullptr;
        uint64_t* xs = nullptr;
        float* w = nullptr;
        int* perm = nullptr;
    } made;
    void* rho = nullptr;        // reduced density matrix (library-owned)
    size_t rho_bytes = 0;
    void* pin = nullptr;        // pinned host staging of pw_eval_states (library-owned)
    size_t pin_bytes = 0;
    void* nrm = nullptr;        // per-state norm slots of pw_eval_states (library-owned)
    size_t nrm_bytes = 0;
    // graph replay of Monte Carlo sampling steps
    bool use_graphs = false;
    hipStream_t gstream = nullptr;  // non-blocking capture stream (default priority)
    hipEvent_t gfork = nullptr, gjoin = nullptr;
    bool capturing = false;
    // error-path testing (pw_inject_fault): the class of HIP call made to fail
    int fault_class = 0;
    // transform arithmetic (pw_set_precision) and what the kernels read: the bound state,
    // or a library-owned copy of it in the compute precision
    int prec = PW_PREC_AUTO;
    bool cdbl = false;           // FP64 kernels (complex128 input)
    bool cmfma = false;          // split-BF16 matrix-core first pass / single-workgroup kernel
    const void* cpsi = nullptr;
    void* conv = nullptr;
    size_t conv_bytes = 0;
    bool conv_valid = false;
    // schedule asked for by pw_set_schedule (zeros: the tuned or default choice)
    Schedule sched{0, 0, 0};
    int sched_batch = 0;
    // progress report of long Monte Carlo runs (pw_set_progress)
    pw_progress_fn progress = nullptr;
    void* progress_user = nullptr;
    double progress_every = 0.0;
};

namespace {

// Forced failure of one class of HIP call (1 allocation, 2 kernel launch, 3 copy) before
// it is issued, set by pw_inject_fault for tests of the error paths.
enum { FAULT_NONE = 0, FAULT_ALLOC = 1, FAULT_LAUNCH = 2, FAULT_COPY = 3 };
inline bool fault(pw_ctx c, int cls) { return c->fault_class == cls; }

// Progress of a long estimate: the callback set by pw_set_progress, at most once per
// progress_every seconds of wall time (always when final).
void report_progress(pw_ctx c, uint64_t families, double M2, double M2_se, bool final) {
    if (!c->progress) return;
    static thread_local std::chrono::steady_clock::time_point last{};
    const auto now = std::chrono::steady_clock::now();
    if (!final && std::chrono::duration<double>(now - last).count() < c->progress_every) return;
    last = now;
    c->progress(c->progress_user, families, M2, M2_se);
}

// Storage dtype of the data the kernels read for a state of storage dtype dt.
pw_dtype compute_dtype(pw_ctx c, pw_dtype dt) {
    if (c->prec == PW_PREC_F64) return PW_C128;
    if (c->prec == PW_PREC_F32 || c->prec == PW_PREC_BF16X2) return PW_C64;
    return dt;
}

// Autotune key of the arithmetic: 0 FP64, 1 FP32, 2 split-BF16.
int prec_key(pw_ctx c, pw_dtype dt) {
    if (c->prec == PW_PREC_BF16X2) return 2;
    return compute_dtype(c, dt) == PW_C128 ? 0 : 1;
}

hipEvent_t take_event(pw_ctx c) {
    if (!c->pool.empty()) {
        hipEvent_t e = c->pool.back();
        c->pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

bool timer_take(void* self, int k, hipEvent_t* a, hipEvent_t* b) {
    pw_ctx c = (pw_ctx)self;
    if (c->launches[k]++ % (uint64_t)c->timing_every != 0) return false;
    hipEvent_t e0 = take_event(c);
    if (!e0) return false;
    hipEvent_t e1 = take_event(c);
    if (!e1) {
        c->pool.push_back(e0);
        return false;
    }
    *a = e0;
    *b = e1;
    return true;
}

void timer_commit(void* self, int k, int families, hipEvent_t a, hipEvent_t b) {
    pw_ctx c = (pw_ctx)self;
    c->pending.push_back({a, b, k, families});
}

const LaunchTimer* timer_of(pw_ctx c) { return (c->timing_every > 0 && !c->capturing) ? &c->timer : nullptr; }

// Autotuned schedules (plan variant, first-pass group, families per launch) per (device,
// n, arithmetic), shared by the contexts of the process; pw_autotune_save / _load keep
// them in a text file.
struct Tuned {
    Schedule sc;
    int batch;
    double us;
};
std::mutex g_tune_mu;
std::map<std::tuple<int, int, int>, Tuned> g_tune;

bool tuned_get(int device, int n, int key, Tuned* t) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune.find(std::make_tuple(device, n, key));
    if (it == g_tune.end()) return false;
    *t = it->second;
    return true;
}

void tuned_put(int device, int n, int key, const Tuned& t) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune[std::make_tuple(device, n, key)] = t;
}

pw_status check_ctx(pw_ctx c) {
    if (!c) return fail(PW_ERR_ARG, "null context");
    return PW_OK;
}

pw_status check_state(pw_ctx c) {
    pw_status s = check_ctx(c);
    if (s != PW_OK) return s;
    if (!c->bound) return fail(PW_ERR_NO_STATE, "no state bound to the context");
    return PW_OK;
}

template <typename T>
T* at(pw_ctx c, size_t off) {
    return reinterpret_cast<T*>(c->ws + off);
}

// Plan and launch size of the bound state: the context's own schedule when it applies,
// else the process's tuned one, else the defaults.
void apply_schedule(pw_ctx c, pw_dtype sdt) {
    const int n = c->n;
    Tuned t{};
    const bool have_tuned = tuned_get(c->device, n, prec_key(c, sdt), &t);
    const bool own = c->sched.first_bits || c->sched.column_tile_bits || c->sched.group;
    Schedule sc = own ? c->sched : (have_tuned ? t.sc : Schedule{0, 0, 0});
    if (c->cmfma) {
        c->P = make_plan_bf16x2(n);
    } else {
        bool ok = true;
        c->P = make_plan_sched(n, c->cdbl, sc, &ok);
    }
    int b = c->sched_batch ? c->sched_batch : (have_tuned ? t.batch : 0);
    c->run_batch = (b > 0 && b < c->batch) ? b : c->batch;
}

// Carve (or allocate) the workspace for the bound state (storage dtype dt): sized and
// planned for the compute precision.
pw_status prepare_workspace(pw_ctx c, int n, pw_dtype sdt) {
    const pw_dtype dt = compute_dtype(c, sdt);
    if (c->ws && !c->ws_owned) {
        int b = MAX_BATCH;
        while (b >= 1 && layout_for(n, dt, b).total > c->ws_bytes) b /= 2;
        if (b < 1)
            return fail(PW_ERR_WORKSPACE, "workspace of %zu bytes is below the %zu needed for n=%d", c->ws_bytes,
                        layout_for(n, dt, 1).total, n);
        c->batch = b;
    } else {
        c->batch = default_batch(n, dt);
        const size_t need = layout_for(n, dt, c->batch).total;
        if (!c->ws || c->ws_bytes < need) {
            if (c->ws) {
                PW_HIP(hipStreamSynchronize(c->stream));
                PW_HIP(hipFree(c->ws));
                c->ws = nullptr;
                c->ws_bytes = 0;
            }
            if (fault(c, FAULT_ALLOC)) return fail(PW_ERR_HIP, "hipMalloc: injected failure");
            void* p = nullptr;
            PW_HIP(hipMalloc(&p, need));
            c->ws = (char*)p;
            c->ws_bytes = need;
            c->ws_owned = true;
        }
    }
    c->L = layout_for(n, dt, c->batch);
    c->cmfma = c->prec == PW_PREC_BF16X2;
    c->cdbl = dt == PW_C128;
    c->cpsi = dt == sdt ? c->psi : nullptr;
    c->conv_valid = dt == sdt;
    apply_schedule(c, sdt);
    return PW_OK;
}

// The state in the compute precision: the bound buffer itself, or a library-owned copy
// converted from it (made again after the state changes).
pw_status ensure_compute_state(pw_ctx c) {
    if (c->conv_valid) return PW_OK;
    const pw_dtype cdt = c->cdbl ? PW_C128 : PW_C64;
    const size_t need = ((size_t)1 << c->n) * esize(cdt);
    if (!c->conv || c->conv_bytes < need) {
        if (c->conv) {
            PW_HIP(hipStreamSynchronize(c->stream));
            PW_HIP(hipFree(c->conv));
            c->conv = nullptr;
            c->conv_bytes = 0;
        }
        if (fault(c, FAULT_ALLOC)) return fail(PW_ERR_HIP, "hipMalloc: injected failure");
        PW_HIP(hipMalloc(&c->conv, need));
        c->conv_bytes = need;
    }
    if (fault(c, FAULT_LAUNCH)) return fail(PW_ERR_HIP, "kernel launch: injected failure");
    PW_HIP(convert_state(c->dtype == PW_C128, c->psi, c->conv, c->n, c->stream));
    c->cpsi = c->conv;
    c->conv_valid = true;
    return PW_OK;
}

pw_status run_norm(pw_ctx c, double* out) {
    const int np = norm2_parts(c->n);
    double* part = at<double>(c, c->L.norm);
    double* res = part + np;
    unsigned* bad = reinterpret_cast<unsigned*>(part + np + 1);
    PW_HIP(hipMemsetAsync(bad, 0, sizeof(unsigned), c->stream));
    if (fault(c, FAULT_LAUNCH)) return fail(PW_ERR_HIP, "kernel launch: injected failure");
    PW_HIP(norm2(c->dtype == PW_C128, c->psi, c->n, part, np, res, bad, c->stream));
    double h[2];
    PW_HIP(hipMemcpyAsync(h, res, 2 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    PW_HIP(hipStreamSynchronize(c->stream));
    unsigned hb;
    memcpy(&hb, &h[1], sizeof hb);
    if (hb) return fail(PW_ERR_NOT_NORMALIZED, "state holds NaN or Inf amplitudes");
    *out = h[0];
    return PW_OK;
}

// Evaluate nx families whose x are in device memory (or x0 + i when d_xs is null),
// results to device array d_out, in launches of the context's launch batch, on st.
pw_status eval_list_on(pw_ctx c, const uint64_t* d_xs, uint64_t x0, int64_t nx, double eps, FamilyRes* d_out,
                       hipStream_t st, const uint64_t* d_fpsi = nullptr) {
    const bool dbl = c->cdbl;
    // multi-pass plans: batches leave their partials side by side, one finalize per group
    const bool defer = !c->P.fused;
    FamilyRes* parts = at<FamilyRes>(c, c->L.parts);
    int64_t g0 = 0, pending = 0;
    for (int64_t i = 0; i < nx; i += c->run_batch) {
        const int nb = (int)((nx - i) < c->run_batch ? (nx - i) : c->run_batch);
        if (defer && pending + nb > c->L.parts_fams) {
            PW_HIP(finalize_families(c->P, c->max_alpha, parts, pending, d_out + g0, st));
            g0 = i;
            pending = 0;
        }
        PW_HIP(eval_batch(c->P, dbl, c->max_alpha, c->cpsi, d_xs ? d_xs + i : nullptr, x0 + (uint64_t)i, nb, eps,
                          c->ws + c->L.work, parts + (size_t)pending * c->P.blocks_last, d_out + i, st,
                          timer_of(c), !defer, d_fpsi ? d_fpsi + i : nullptr));
        pending += nb;
    }
    if (defer && pending > 0) PW_HIP(finalize_families(c->P, c->max_alpha, parts, pending, d_out + g0, st));
    return PW_OK;
}

pw_status eval_device_on(pw_ctx c, const uint64_t* d_xs, uint64_t x0, int64_t nx, double eps, FamilyRes* d_out,
                         hipStream_t st) {
    if (fault(c, FAULT_LAUNCH)) return fail(PW_ERR_HIP, "kernel launch: injected failure");
    const pw_status sc = ensure_compute_state(c);
    if (sc != PW_OK) return sc;
    if (!d_xs || first_pass_group(c->P, c->cdbl, c->run_batch) < 2)
        return eval_list_on(c, d_xs, x0, nx, eps, d_out, st);
    // tile-sharing groups: the list is evaluated in top-bit order, so that the families
    // of a launch share state tiles, and the results are put back in list order
    uint64_t* xs2 = at<uint64_t>(c, c->L.xsort);
    uint32_t* perm = at<uint32_t>(c, c->L.perm);
    FamilyRes* r2 = at<FamilyRes>(c, c->L.xres2);
    for (int64_t i = 0; i < nx; i += c->L.xcap) {
        const int m = (int)((nx - i) < c->L.xcap ? (nx - i) : c->L.xcap);
        PW_HIP(sort_by_top_bit(d_xs + i, c->n, m, xs2, perm, st));
        const pw_status s = eval_list_on(c, xs2, 0, m, eps, r2, st);
        if (s != PW_OK) return s;
        PW_HIP(scatter_results(r2, perm, m, d_out + i, st));
    }
    return PW_OK;
}

pw_status eval_device(pw_ctx c, const uint64_t* d_xs, uint64_t x0, int64_t nx, double eps, FamilyRes* d_out) {
    return eval_device_on(c, d_xs, x0, nx, eps, d_out, c->stream);
}

pw_status eval_host(pw_ctx c, const uint64_t* xs, int64_t nx, double eps, FamilyRes* out) {
    uint64_t* dx = at<uint64_t>(c, c->L.xs);
    FamilyRes* dr = at<FamilyRes>(c, c->L.xres);
    for (int64_t i = 0; i < nx; i += c->L.xcap) {
        const int nb = (int)((nx - i) < c->L.xcap ? (nx - i) : c->L.xcap);
        if (fault(c, FAULT_COPY)) return fail(PW_ERR_HIP, "hipMemcpy: injected failure");
        PW_HIP(hipMemcpyAsync(dx, xs + i, nb * sizeof(uint64_t), hipMemcpyHostToDevice, c->stream));
        pw_status s = eval_device(c, dx, 0, nb, eps, dr);
        if (s != PW_OK) return s;
        PW_HIP(hipMemcpyAsync(out + i, dr, nb * sizeof(FamilyRes), hipMemcpyDeviceToHost, c->stream));
        PW_HIP(hipStreamSynchronize(c->stream));
    }
    return PW_OK;
}

bool is_pow2(uint64_t v) { return v && !(v & (v - 1)); }

// Welford running mean / variance (fixed order, so reproducible).
struct Running {
    double n = 0, mean = 0, m2 = 0;
    void add(double y) {
        n += 1;
        const double d = y - mean;
        mean += d / n;
        m2 += d * (y - mean);
    }
    double var() const { return n > 1 ? m2 / (n - 1) : NAN; }
};

// Graph replay of one Monte Carlo step: draw `nb` x on the device (counters start at
// the device counter), evaluate their families into the per-family buffer, advance the
// counter.  The step is captured once on a private non-blocking stream and replayed;
// it records no memset or copy nodes.
struct McGraph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipStream_t st = nullptr;  // the replay stream; drained first, so that a call that
                               // fails between replays leaves no step running
    ~McGraph() {
        if (exec && st) (void)hipStreamSynchronize(st);
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
    }
};

pw_status mc_step_enqueue(pw_ctx c, pw_sampler sampler, uint64_t seed, int nb, double eps, hipStream_t st) {
    uint64_t* dx = at<uint64_t>(c, c->L.xs);
    uint64_t* dctr = at<uint64_t>(c, c->L.ctr);
    if (sampler == PW_SAMPLER_UNIFORM_NZ) PW_HIP(sample_uniform(c->n, seed, 0, nb, dx, st, dctr));
    else PW_HIP(sample_marginal(c->n, at<double>(c, c->L.cdf), seed, 0, nb, dx, st, dctr));
    // the families in chunks of the launch batch
    const pw_status s = eval_device_on(c, dx, 0, nb, eps, at<FamilyRes>(c, c->L.xres), st);
    if (s != PW_OK) return s;
    PW_HIP(bump_counter(dctr, (uint64_t)nb, st));
    return PW_OK;
}

pw_status mc_graph_build(pw_ctx c, pw_sampler sampler, uint64_t seed, int nb, double eps, McGraph& g) {
    if (!c->gstream) {
        PW_HIP(hipStreamCreateWithFlags(&c->gstream, hipStreamNonBlocking));
        PW_HIP(hipEventCreateWithFlags(&c->gfork, hipEventDisableTiming));
        PW_HIP(hipEventCreateWithFlags(&c->gjoin, hipEventDisableTiming));
    }
    c->capturing = true;
    hipError_t e = hipStreamBeginCapture(c->gstream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
        c->capturing = false;
        return fail(PW_ERR_HIP, "hipStreamBeginCapture: %s", hipGetErrorString(e));
    }
    pw_status s = mc_step_enqueue(c, sampler, seed, nb, eps, c->gstream);
    e = hipStreamEndCapture(c->gstream, &g.graph);
    c->capturing = false;
    if (s != PW_OK) return s;
    if (e != hipSuccess) return fail(PW_ERR_HIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
    PW_HIP(hipGraphInstantiate(&g.exec, g.graph, nullptr, nullptr, 0));
    g.st = c->gstream;
    return PW_OK;
}

}  // namespace

extern "C" {

const char* pw_last_error(void) { return g_err.c_str(); }

const char* pw_version(void) { return "pauliwht 0.1 (gfx950)"; }

pw_status pw_ctx_create(pw_ctx* out, int device, void* hip_stream) {
    if (!out) return fail(PW_ERR_ARG, "null output pointer");
    if (device < 0) return fail(PW_ERR_ARG, "negative device index");
    PW_HIP(hipSetDevice(device));
    pw_ctx c = new pw_ctx_s();
    c->device = device;
    c->stream = (hipStream_t)hip_stream;
    c->timer.take = timer_take;
    c->timer.commit = timer_commit;
    c->timer.self = c;
    *out = c;
    g_err.clear();
    return PW_OK;
}

pw_status pw_ctx_destroy(pw_ctx c) {
    if (!c) return fail(PW_ERR_ARG, "null context");
    pw_status s = PW_OK;
    (void)hipStreamSynchronize(c->stream);
    for (auto& p : c->pending) {
        (void)hipEventDestroy(p.a);
        (void)hipEventDestroy(p.b);
    }
    for (auto e : c->pool) (void)hipEventDestroy(e);
    if (c->made.block) (void)hipFree(c->made.block);
    if (c->rho) (void)hipFree(c->rho);
    if (c->conv) (void)hipFree(c->conv);
    if (c->pin) (void)hipHostFree(c->pin);
    if (c->nrm) (void)hipFree(c->nrm);
    if (c->gstream) {
        (void)hipStreamSynchronize(c->gstream);
        (void)hipStreamDestroy(c->gstream);
    }
    if (c->gfork) (void)hipEventDestroy(c->gfork);
    if (c->gjoin) (void)hipEventDestroy(c->gjoin);
    if (c->ws && c->ws_owned) {
        if (hipStreamSynchronize(c->stream) != hipSuccess || hipFree(c->ws) != hipSuccess)
            s = fail(PW_ERR_HIP, "releasing the library-owned workspace failed");
    }
    delete c;
    return s;
}

pw_status pw_workspace_size(int n, pw_dtype dt, int x_batch, size_t* bytes) {
    if (!bytes) return fail(PW_ERR_ARG, "null output pointer");
    if (dt != PW_C128 && dt != PW_C64) return fail(PW_ERR_ARG, "unknown dtype %d", (int)dt);
    if (n < 1 || n > MAX_QUBITS) return fail(PW_ERR_RANGE, "n=%d outside [1, %d]", n, MAX_QUBITS);
    if (x_batch < 1 || x_batch > MAX_BATCH) return fail(PW_ERR_RANGE, "x_batch=%d outside [1, %d]", x_batch, MAX_BATCH);
    *bytes = layout_for(n, dt, x_batch).total;
    return PW_OK;
}

pw_status pw_set_workspace(pw_ctx c, void* dev, size_t bytes) {
    pw_status s = check_ctx(c);
    if (s != PW_OK) return s;
    if (dev && ((uintptr_t)dev & 255)) return fail(PW_ERR_ARG, "workspace must be 256-byte aligned");
    if (c->ws && c->ws_owned) {
        PW_HIP(hipStreamSynchronize(c->stream));
        PW_HIP(hipFree(c->ws));
    }
    c->ws = (char*)dev;
    c->ws_bytes = dev ? bytes : 0;
    c->ws_owned = false;
    if (c->bound) {
        c->bound = false;   // re-carve on the next bind
        c->cdf_valid = false;
        if (dev) {
            s = prepare_workspace(c, c->n, c->dtype);
            if (s != PW_OK) return s;
            c->bound = true;
        }
    }
    return PW_OK;
}

pw_status pw_state_bind(pw_ctx c, int n, pw_dtype dt, void* dev_psi, double* norm2_out) {
    pw_status s = check_ctx(c);
    if (s != PW_OK) return s;
    if (!dev_psi) return fail(PW_ERR_ARG, "null state pointer");
    if ((uintptr_t)dev_psi & 255) return fail(PW_ERR_ARG, "state must be 256-byte aligned");
    if (dt != PW_C128 && dt != PW_C64) return fail(PW_ERR_ARG, "unknown dtype %d", (int)dt);
    if (n < 1 || n > MAX_QUBITS) return fail(PW_ERR_RANGE, "n=%d outside [1, %d]", n, MAX_QUBITS);
    c->bound = false;
    c->cdf_valid = false;
    c->psi = dev_psi;
    c->n = n;
    c->dtype = dt;
    s = prepare_workspace(c, n, dt);
    if (s != PW_OK) return s;
    double nrm = 0.0;
    s = run_norm(c, &nrm);
    if (s != PW_OK) return s;
    const double tol = dt == PW_C128 ? 1e-10 : 1e-5;
    if (!(fabs(nrm - 1.0) <= tol))
        return fail(PW_ERR_NOT_NORMALIZED, "<psi|psi> = %.17g differs from 1 by more than %g", nrm, tol);
    c->bound = true;
    if (norm2_out) *norm2_out = nrm;
    return PW_OK;
}

pw_status pw_state_upload(pw_ctx c, int n, pw_dtype dt, const void* host_psi, void* dev_dst, double* norm2_out) {
    pw_status s = check_ctx(c);
    if (s != PW_OK) return s;
    if (!host_psi || !dev_dst) return fail(PW_ERR_ARG, "null pointer");
    if (dt != PW_C128 && dt != PW_C64) return fail(PW_ERR_ARG, "unknown dtype %d", (int)dt);
    if (n < 1 || n > MAX_QUBITS) return fail(PW_ERR_RANGE, "n=%d outside [1, %d]", n, MAX_QUBITS);
    if (fault(c, FAULT_COPY)) return fail(PW_ERR_HIP, "hipMemcpy: injected failure");
    PW_HIP(hipMemcpyAsync(dev_dst, host_psi, ((size_t)1 << n) * esize(dt), hipMemcpyHostToDevice, c->stream));
    return pw_state_bind(c, n, dt, dev_dst, norm2_out);
}

pw_status pw_apply_gates(pw_ctx c, int ng, const int* kinds, const int* qubits, const double* mats) {
    pw_status s = check_state(c);
    if (s != PW_OK) return s;
    if (ng < 0) return fail(PW_ERR_ARG, "negative gate count");
    if (ng > 0 && (!kinds || !qubits || !mats)) return fail(PW_ERR_ARG, "null gate array");
    for (int g = 0; g < ng; ++g) {
        const int q0 = qubits[2 * g], q1 = qubits[2 * g + 1];
        if (kinds[g] == 2) {
            if (c->n < 2 || q0 < 0 || q1 < 0 || q0 >= c->n || q1 >= c->n || q0 == q1)
                return fail(PW_ERR_RANGE, "gate %d: qubits (%d, %d) invalid for n=%d", g, q0, q1, c->n);
        } else if (kinds[g] == 1) {
            if (q0 < 0 || q0 >= c->n) return fail(PW_ERR_RANGE, "gate %d: qubit %d invalid for n=%d", g, q0, c->n);
        } else {
            return fail(PW_ERR_ARG, "gate %d: unknown kind %d", g, kinds[g]);
        }
    }
    if (fault(c, FAULT_LAUNCH)) return fail(PW_ERR_HIP, "kernel launch: injected failure");
    const bool dbl = c->dtype == PW_C128;
    for (int g = 0; g < ng; ++g) {
        if (kinds[g] == 2) PW_HIP(apply_gate2(dbl, c->psi, c->n, qubits[2 * g], qubits[2 * g + 1], mats + 32 * g, c->stream));
        else PW_HIP(apply_diag(dbl, c->psi, c->n, qubits[2 * g], mats + 32 * g, c->stream));
    }
    c->cdf_valid = false;
    c->conv_valid = c->cpsi == c->psi;
    PW_HIP(hipStreamSynchronize(c->stream));
    return PW_OK;
}

pw_status pw_clifford2_table(int* count, double* mats) {
    const int m = clifford2_count();
    if (count) *count = m;
    if (mats)
        for (int i = 0; i < m; ++i) clifford2_matrix(i, mats + 32 * (size_t)i);
    return PW_OK;
}

pw_status pw_precondition_circuit(int n, int n_layers, uint64_t seed, int64_t* n_gates, int* qubits, double* mats) {
    if (n < 2 || n > MAX_QUBITS) return fail(PW_ERR_RANGE, "n=%d outside [2, %d]", n, MAX_QUBITS);
    if (n_layers < 0) return fail(PW_ERR_ARG, "negative layer count");
    std::vector<int> q, idx;
    brickwall_clifford(n, n_layers, seed, q, idx);
    if (n_gates) *n_gates = (int64_t)idx.size();
    for (size_t g = 0; g < idx.size(); ++g) {
        if (qubits) {
            qubits[2 * g] = q[2 * g];
            qubits[2 * g + 1] = q[2 * g + 1];
        }
        if (mats) clifford2_matrix(idx[g], mats + 32 * g);
    }
    return PW_OK;
}

pw_status pw_precondition(pw_ctx c, int n_layers, uint64_t seed) {
    pw_status s = check_state(c);
    if (s != PW_OK) return s;
    if (c->n < 2) return fail(PW_ERR_RANGE, "preconditioning needs n >= 2");
    if (n_layers < 0) return fail(PW_ERR_ARG, "negative layer count");
    if (fault(c, FAULT_LAUNCH)) return fail(PW_ERR_HIP, "kernel launch: injected failure");
    std::vector<int> q, idx, ls;
    brickwall_clifford(c->n, n_layers, seed, q, idx, &ls);
    ls.push_back((int)idx.size());
    const bool dbl = c->dtype == PW_C128;
    const int n = c->n;
    // The gates of a layer act on disjoint pairs (they commute) and are grouped into
    // passes over LDS tiles: one tile of the low 12 bits, then windows of bits [0, 4)
    // and [hb, hb + 8) that cover the remaining pairs (see apply_gates_tile).
    auto apply_group = [&](const std::vector<int>& gs, int W, int hb, int H) -> hipError_t {
        int a[6], b[6];
        double m32[6 * 32];
        int k = 0;
        for (int g : gs) {
            auto local = [&](int qb) { return qb < W ? qb : W + (qb - hb); };
            a[k] = local(q[2 * g]);
            b[k] = local(q[2 * g + 1]);
            clifford2_matrix(idx[g], m32 + 32 * k);
            if (++k == 6) {
                hipError_t e = apply_gates_tile(dbl, c->psi, n, W, hb, H, k, a, b, m32, c->stream);
                if (e != hipSuccess) return e;
                k = 0;
            }
        }
        return k ? apply_gates_tile(dbl, c->psi, n, W, hb, H, k, a, b, m32, c->stream) : hipSuccess;
    };
    for (size_t l = 0; l + 1 < ls.size(); ++l) {
        std::vector<int> rem;
        for (int g = ls[l]; g < ls[l + 1]; ++g) rem.push_back(g);
        if (n <= 12) {
            PW_HIP(apply_group(rem, n, n, 0));
            continue;
        }
        auto in_tile = [&](int qb, int W, int hb, int H) { return qb < W || (H > 0 && qb >= hb && qb < hb + H); };
        std::vector<int> first, rest;
        for (int g : rem) (q[2 * g] < 12 && q[2 * g + 1] < 12 ? first : rest).push_back(g);
        if (!first.empty()) PW_HIP(apply_group(first, 12, 12, 0));
        while (!rest.empty()) {
            int m = n;
            for (int g : rest)
                for (int j = 0; j < 2; ++j)
                    if (q[2 * g + j] >= 4 && q[2 * g + j] < m) m = q[2 * g + j];
            const int hb = m < n - 8 ? m : n - 8;
            std::vector<int> take, left;
            for (int g : rest)
                (in_tile(q[2 * g], 4, hb, 8) && in_tile(q[2 * g + 1], 4, hb, 8) ? take : left).push_back(g);
            if (take.empty()) {
                // not reached for brick-wall pairs; a pair the windows cannot hold goes alone
                const int g = rest.front();
                double m32[32];
                clifford2_matrix(idx[g], m32);
                PW_HIP(apply_gate2(dbl, c->psi, n, q[2 * g], q[2 * g + 1], m32, c->stream));
                left.assign(rest.begin() + 1, rest.end());
            } else {
                PW_HIP(apply_group(take, 4, hb, 8));
            }
            rest.swap(left);
        }
    }
    c->cdf_valid = false;
    c->conv_valid = c->cpsi == c->psi;
    PW_HIP(hipStreamSynchronize(c->stream));
    return PW_OK;
}

pw_status pw_eval_x(pw_ctx c, const uint64_t* xs, int64_t nx, double eps, pw_xres* out) {
    pw_status s = check_state(c);
    if (s != PW_OK) return s;
    if (nx < 0) return fail(PW_ERR_ARG, "negative count");
    if (nx > 0 && (!xs || !out)) return fail(PW_ERR_ARG, "null array");
    if (!(eps >= 0.0 && eps < 1.0)) return fail(PW_ERR_ARG, "eps=%g outside [0, 1)", eps);
    const uint64_t d = 1ull << c->n;
    for (int64_t i = 0; i < nx; ++i)
        if (xs[i] >= d) return fail(PW_ERR_RANGE, "xs[%lld] = %llu is not below 2^%d", (long long)i, (unsigned long long)xs[i], c->n);
    std::vector<FamilyRes> tmp((size_t)nx);
    s = eval_host(c, xs, nx, eps, tmp.data());
    if (s != PW_OK) return s;
    memcpy(out, tmp.data(), (size_t)nx * sizeof(FamilyRes));
    return PW_OK;
}

pw_status pw_eval_x_device(pw_ctx c, const uint64_t* d_xs, int64_t nx, double eps, pw_xres* d_out) {
    pw_status s = check_state(c);
    if (s != PW_OK) return s;
    if (nx < 0) return fail(PW_ERR_ARG, "negative count");
    if (nx > 0 && (!d_xs || !d_out)) return fail(PW_ERR_ARG, "null array");
    if (!(eps >= 0.0 && eps < 1.0)) return fail(PW_ERR_ARG, "eps=%g outside [0, 1)", eps);
    return eval_device(c, d_xs, 0, nx, eps, reinterpret_cast<FamilyRes*>(d_out));
}

pw_status pw_family_values(pw_ctx c, uint64_t x, double* cvals) {
    pw_status s = check_state(c);
    if (s != PW_OK) return s;
    if (!cvals) return fail(PW_ERR_ARG, "null output");
    if (c->n > FAMILY_VALUES_MAX_QUBITS) return fail(PW_ERR_RANGE, "family values limited to n <= %d", FAMILY_VALUES_MAX_QUBITS);
    if (x >= (1ull << c->n)) return fail(PW_ERR_RANGE, "x not below 2^n");
    const bool dbl = c->dtype == PW_C128;
    void* G = c->ws + c->L.work;
    double* cv = reinterpret_cast<double*>(c->ws + c->L.work + align256(((size_t)1 << (c->n - 1)) * esize(c->dtype)));
    Plan P = make_plan(c->n, dbl);
    if (fault(c, FAULT_LAUNCH)) return fail(PW_ERR_HIP, "kernel launch: injected failure");
    PW_HIP(transform_one(P, dbl, c->psi, x, G, c->stream));
    PW_HIP(signed_values(P, dbl, G, x, cv, c->stream));
    PW_HIP(hipMemcpyAsync(cvals, cv, ((size_t)1 << c->n) * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    PW_HIP(hipStreamSynchronize(c->stream));
    return PW_OK;
}

pw_status pw_sample_x(pw_ctx c, pw_sampler sampler, uint64_t seed, uint64_t offset, int64_t n, uint64_t* xs_out) {
    pw_status s = check_state(c);
    if (s != PW_OK) return s;
    if (n < 0) return fail(PW_ERR_ARG, "negative count");
    if (n > 0 && !xs_out) return fail(PW_ERR_ARG, "null output");
    if (sampler != PW_SAMPLER_UNIFORM_NZ && sampler != PW_SAMPLER_MARGINAL_NZ) return fail(PW_ERR_ARG, "unknown sampler");
    if (c->n < 1) return fail(PW_ERR_RANGE, "need n >= 1");
    if (fault(c, FAULT_LAUNCH)) return fail(PW_ERR_HIP, "kernel launch: injected failure");
    uint64_t* dx = at<uint64_t>(c, c->L.xs);
    if (sampler == PW_SAMPLER_MARGINAL_NZ && !c->cdf_valid) {
        PW_HIP(build_cdf(c->dtype == PW_C128, c->psi, c->n, at<double>(c, c->L.cdf), at<double>(c, c->L.cdfblk), c->stream));
        c->cdf_valid = true;
    }
    for (int64_t i = 0; i < n; i += c->L.xcap) {
        const int64_t nb = (n - i) < c->L.xcap ? (n - i) : c->L.xcap;
        if (sampler == PW_SAMPLER_UNIFORM_NZ) PW_HIP(sample_uniform(c->n, seed, offset + (uint64_t)i, nb, dx, c->stream));
        else PW_HIP(sample_marginal(c->n, at<double>(c, c->L.cdf), seed, offset + (uint64_t)i, nb, dx, c->stream));
        PW_HIP(hipMemcpyAsync(xs_out + i, dx, nb * sizeof(uint64_t), hipMemcpyDeviceToHost, c->stream));
        PW_HIP(hipStreamSynchronize(c->stream));
    }
    return PW_OK;
}

pw_status pw_exact(pw_ctx c, double eps, pw_result* out) {
    pw_status s = check_state(c);
    if (s != PW_OK) return s;
    if (!out) return fail(PW_ERR_ARG, "null output");
    if (!(eps >= 0.0 && eps < 1.0)) return fail(PW_ERR_ARG, "eps=%g outside [0, 1)", eps);
    if (c->n > EXACT_MAX_QUBITS) return fail(PW_ERR_RANGE, "exact enumeration limited to n <= %d", EXACT_MAX_QUBITS);
    if (fault(c, FAULT_LAUNCH)) return fail(PW_ERR_HIP, "kernel launch: injected failure");
    const uint64_t d = 1ull << c->n;
    SweepSums* sw = at<SweepSums>(c, c->L.sweep);
    SweepSums* fin = sw + SWEEP_SLOTS;
    FamilyRes* fam = at<FamilyRes>(c, c->L.fam);
    int64_t nchunk = 0;
    for (uint64_t c0 = 0; c0 < d; c0 += (uint64_t)EXACT_CHUNK) {
        const int64_t cnt = (int64_t)((d - c0) < (uint64_t)EXACT_CHUNK ? (d - c0) : (uint64_t)EXACT_CHUNK);
        s = eval_device(c, nullptr, c0, cnt, eps, fam);
        if (s != PW_OK) return s;
        if (nchunk + reduce_families_slots(cnt) > SWEEP_SLOTS) return fail(PW_ERR_UNSUPPORTED, "too many chunks");
        PW_HIP(reduce_families(fam, cnt, sw + nchunk, c->stream));
        nchunk += reduce_families_slots(cnt);
    }
    PW_HIP(reduce_sweep(sw, nchunk, fin, c->stream));
    SweepSums h;
    PW_HIP(hipMemcpyAsync(&h, fin, sizeof h, hipMemcpyDeviceToHost, c->stream));
    PW_HIP(hipStreamSynchronize(c->stream));
    pw_result r;
    memset(&r, 0, sizeof r);
    const int n = c->n;
    for (int a = 0; a < 3; ++a) {
        r.S[a] = h.S[a];
        r.S_se[a] = 0.0;
        r.M[a] = log2(h.S[a]) / (1.0 - (a + 2)) - n;
        r.M_se[a] = 0.0;
        // r_alpha = Std_{x != 0}(m_{alpha;x}) / E_x[m_{alpha;x}] (population spread over
        // the d - 1 families x != 0, mean over all d families)
        const double dm1 = (double)(d - 1);
        const double mean_nz = h.Snz[a] / dm1;
        const double var = fmax(h.Q[a] / dm1 - mean_nz * mean_nz, 0.0);
        r.r[a] = d > 1 ? sqrt(var) / (h.S[a] / (double)d) : NAN;
    }
    r.L = h.L;
    r.L_se = 0.0;
    r.M1 = -ldexp(h.L, -n);
    r.M1_se = 0.0;
    r.P = h.P;
    r.nu_cnt = h.nu_cnt;
    r.nullity = h.nu_cnt ? n - log2((double)h.nu_cnt) : NAN;
    r.n_samples = h.count;
    r.gap = h.gap;
    *out = r;
    if (!is_pow2(h.nu_cnt))
        return fail(PW_ERR_TOLERANCE, "nullity count %llu is not a power of two (gap %.3g): eps does not separate |c| = 1",
                    (unsigned long long)h.nu_cnt, h.gap);
    return PW_OK;
}

namespace {
struct DrawMP {
    double m2, p;
};
pw_status mc_core(pw_ctx c, pw_sampler sampler, double eps, int batch, uint64_t max_samples, double target_se,
                  uint64_t seed, pw_result* out, std::vector<DrawMP>* draws);
}

pw_status pw_mc(pw_ctx c, pw_sampler sampler, double eps, int batch, uint64_t max_samples, double target_se,
                uint64_t seed, pw_result* out) {
    return mc_core(c, sampler, eps, batch, max_samples, target_se, seed, out, nullptr);
}

namespace {
// The estimator of pw_mc; with draws != nullptr each drawn family's m_{2;x} and p(x) are
// also returned (the pilot of pw_mc_auto).
pw_status mc_core(pw_ctx c, pw_sampler sampler, double eps, int batch, uint64_t max_samples, double target_se,
                  uint64_t seed, pw_result* out, std::vector<DrawMP>* draws) {
    pw_status s = check_state(c);
    if (s != PW_OK) return s;
    if (!out) return fail(PW_ERR_ARG, "null output");
    if (sampler != PW_SAMPLER_UNIFORM_NZ && sampler != PW_SAMPLER_MARGINAL_NZ) return fail(PW_ERR_ARG, "unknown sampler");
    if (batch < 1) return fail(PW_ERR_ARG, "batch must be >= 1");
    if (max_samples < 3) return fail(PW_ERR_ARG, "max_samples must be >= 3");
    if (!(eps >= 0.0 && eps < 1.0)) return fail(PW_ERR_ARG, "eps=%g outside [0, 1)", eps);
    const int n = c->n;
    const double d = ldexp(1.0, n);
    // x = 0 is always evaluated (Monte Carlo section).
    FamilyRes r0;
    const uint64_t zero = 0;
    s = eval_host(c, &zero, 1, eps, &r0);
    if (s != PW_OK) return s;
    const double p0 = r0.p;
    if (sampler == PW_SAMPLER_MARGINAL_NZ && !(p0 < 1.0 - 1e-12))
        return fail(PW_ERR_UNSUPPORTED, "p(0) = %.17g: the x-marginal has no mass on x != 0", p0);
    Running run[4];   // alpha = 2, 3, 4 and the Shannon term
    double gap = r0.gap;
    uint64_t drawn = 0;
    std::vector<uint64_t> xs;
    std::vector<FamilyRes> res;
    const uint64_t draws_max = max_samples - 1;
    int batches = 0;
    const bool graphs = c->use_graphs && batch <= c->L.xcap;
    McGraph g;
    if (graphs) {
        if (sampler == PW_SAMPLER_MARGINAL_NZ && !c->cdf_valid) {
            PW_HIP(build_cdf(c->dtype == PW_C128, c->psi, c->n, at<double>(c, c->L.cdf), at<double>(c, c->L.cdfblk),
                             c->stream));
            c->cdf_valid = true;
        }
        s = mc_graph_build(c, sampler, seed, batch, eps, g);
        if (s != PW_OK) return s;
        const uint64_t zero64 = 0;
        PW_HIP(hipMemcpyAsync(at<uint64_t>(c, c->L.ctr), &zero64, sizeof zero64, hipMemcpyHostToDevice, c->stream));
        PW_HIP(hipEventRecord(c->gfork, c->stream));
        PW_HIP(hipStreamWaitEvent(c->gstream, c->gfork, 0));
    }
    while (drawn < draws_max) {
        const int64_t nb = (int64_t)((draws_max - drawn) < (uint64_t)batch ? (draws_max - drawn) : (uint64_t)batch);
        xs.resize((size_t)nb);
        res.resize((size_t)nb);
        if (graphs && nb == batch) {
            PW_HIP(hipGraphLaunch(g.exec, c->gstream));
            PW_HIP(hipMemcpyAsync(res.data(), at<FamilyRes>(c, c->L.xres), (size_t)nb * sizeof(FamilyRes),
                                  hipMemcpyDeviceToHost, c->gstream));
            PW_HIP(hipStreamSynchronize(c->gstream));
            for (int64_t i = 0; i < nb; ++i) xs[i] = res[i].x;
        } else {
            if (graphs) PW_HIP(hipStreamSynchronize(c->gstream));
            s = pw_sample_x(c, sampler, seed, drawn, nb, xs.data());
            if (s != PW_OK) return s;
            for (int64_t i = 0; i < nb; ++i)
                if (xs[i] == 0) return fail(PW_ERR_UNSUPPORTED, "the marginal sampler drew x = 0 (|psi|^2 is a point mass)");
            s = eval_host(c, xs.data(), nb, eps, res.data());
            if (s != PW_OK) return s;
        }
        for (int64_t i = 0; i < nb; ++i) {
            if (xs[i] == 0) return fail(PW_ERR_UNSUPPORTED, "the marginal sampler drew x = 0 (|psi|^2 is a point mass)");
            const FamilyRes& f = res[i];
            const double w = sampler == PW_SAMPLER_UNIFORM_NZ ? (d - 1.0) : (1.0 - p0) / f.p;
            for (int a = 0; a < 3; ++a) run[a].add(w * f.m[a]);
            if (draws) draws->push_back({f.m[0], f.p});
            run[3].add(w * f.ent);
            gap = fmax(gap, f.gap);
        }
        drawn += (uint64_t)nb;
        ++batches;
        const double S2 = r0.m[0] + run[0].mean;
        const double se2 = sqrt(run[0].var() / run[0].n);
        const double Mse = se2 / (log(2.0) * S2);
        report_progress(c, drawn + 1, -log2(S2) - n, Mse, false);
        if (batches >= 2 && target_se > 0 && Mse <= target_se) break;
    }
    if (graphs) {
        PW_HIP(hipEventRecord(c->gjoin, c->gstream));
        PW_HIP(hipStreamWaitEvent(c->stream, c->gjoin, 0));
    }
    pw_result r;
    memset(&r, 0, sizeof r);
    for (int a = 0; a < 3; ++a) {
        const double S = r0.m[a] + run[a].mean;
        const double se = sqrt(run[a].var() / run[a].n);
        r.S[a] = S;
        r.S_se[a] = se;
        r.M[a] = log2(S) / (1.0 - (a + 2)) - n;
        r.M_se[a] = se / (fabs(1.0 - (a + 2)) * log(2.0) * S);
        r.r[a] = sqrt(run[a].var()) / S;
    }
    r.L = r0.ent + run[3].mean;
    r.L_se = sqrt(run[3].var() / run[3].n);
    r.M1 = -r.L / d;
    r.M1_se = r.L_se / d;
    r.P = NAN;
    r.nullity = NAN;
    r.nu_cnt = 0;
    r.n_samples = drawn + 1;
    r.gap = gap;
    *out = r;
    return PW_OK;
}

// Relative spreads r = sd(y)/S of both samplers' per-draw terms (alpha = 2), from one
// pilot of exact-marginal draws x_i ~ p(x | x != 0).  The marginal's terms are
// y = (1 - p0) m_x / p(x) directly.  The uniform sampler's terms (d - 1) m_x have mean
// S - m_0 as well, and second moment
//     sum_{x != 0} (d - 1) m_x^2 = E_marginal[ (d - 1) (1 - p0) m_x^2 / p(x) ],
// estimated from the same draws.  Since m_x <= p(x)/d (|F| <= 1), the marginal draws weight
// every x by at least its share of that moment, so the rare families with large m_x that
// dominate the uniform sampler's variance (and that a short uniform pilot usually misses)
// are the ones the marginal draws most often.
struct Spreads {
    double r_uniform, r_marginal;
};
Spreads spreads_from_marginal_pilot(const std::vector<DrawMP>& v, double m0, double p0, double d) {
    const double n = (double)v.size();
    double sy = 0.0, syy = 0.0, su2 = 0.0;
    for (const DrawMP& t : v) {
        const double y = (1.0 - p0) * t.m2 / t.p;
        sy += y;
        syy += y * y;
        su2 += (d - 1.0) * y * t.m2;
    }
    const double mu = sy / n;
    const double S = m0 + mu;
    Spreads sp;
    sp.r_marginal = sqrt(fmax(syy / n - mu * mu, 0.0) * n / (n - 1.0)) / S;
    sp.r_uniform = sqrt(fmax(su2 / n - mu * mu, 0.0) * n / (n - 1.0)) / S;
    return sp;
}
}  // namespace

pw_status pw_mc_auto(pw_ctx c, double eps, int batch, uint64_t max_samples, double target_se, uint64_t seed,
                     int64_t pilot, pw_sampler* chosen, double* pilot_r2, pw_result* out) {
    pw_status s = check_state(c);
    if (s != PW_OK) return s;
    if (!out) return fail(PW_ERR_ARG, "null output");
    if (pilot < 2) return fail(PW_ERR_ARG, "pilot must be >= 2 draws");
    // pilot estimates of both samplers on their own Philox streams (keyed seed ^ "PILOT" + k),
    // so that the estimate that follows draws independently of the choice
    // one pilot of exact-marginal draws on its own Philox stream (key seed ^ "PILOT"), so that
    // the estimate that follows draws independently of the choice
    double r2[2] = {NAN, NAN};
    const uint64_t pseed = seed ^ 0x50494C4F54ull;
    std::vector<DrawMP> v;
    pw_result pr;
    s = mc_core(c, PW_SAMPLER_MARGINAL_NZ, eps, batch, (uint64_t)pilot + 1, 0.0, pseed, &pr, &v);
    if (s == PW_OK) {
        FamilyRes r0;
        const uint64_t zero = 0;
        s = eval_host(c, &zero, 1, eps, &r0);
        if (s != PW_OK) return s;
        const Spreads sp = spreads_from_marginal_pilot(v, r0.m[0], r0.p, ldexp(1.0, c->n));
        r2[0] = sp.r_uniform;
        r2[1] = sp.r_marginal;
    } else if (s != PW_ERR_UNSUPPORTED) {
        return s;   // PW_ERR_UNSUPPORTED: no mass on x != 0, only the uniform sampler runs
    }
    // the sample count for a target error grows as r_2^2 (Eq. stdM): the smaller spread wins
    const pw_sampler pick = (r2[1] < r2[0]) ? PW_SAMPLER_MARGINAL_NZ : PW_SAMPLER_UNIFORM_NZ;
    s = pw_mc(c, pick, eps, batch, max_samples, target_se, seed, out);
    if (s != PW_OK) return s;
    if (chosen) *chosen = pick;
    if (pilot_r2) {
        pilot_r2[0] = r2[0];
        pilot_r2[1] = r2[1];
    }
    return PW_OK;
}

// ---------------------------------------------------------------------------
// Learned proposal
// ---------------------------------------------------------------------------

namespace {

constexpr int MADE_MAXB = 4096;

pw_status made_check(pw_ctx c) {
    pw_status s = check_ctx(c);
    if (s != PW_OK) return s;
    if (!c->made.ready) return fail(PW_ERR_NO_STATE, "no learned proposal: call pw_made_init first");
    return PW_OK;
}

// Upload up to MADE_MAXB x values (and weights) to the MADE staging buffers.
pw_status made_stage(pw_ctx c, const uint64_t* xs, const double* w, int64_t count) {
    auto& M = c->made;
    PW_HIP(hipMemcpyAsync(M.xs, xs, (size_t)count * sizeof(uint64_t), hipMemcpyHostToDevice, c->stream));
    if (w) {
        std::vector<float> wf((size_t)count);
        for (int64_t i = 0; i < count; ++i) wf[i] = (float)w[i];
        PW_HIP(hipMemcpyAsync(M.w, wf.data(), (size_t)count * sizeof(float), hipMemcpyHostToDevice, c->stream));
        PW_HIP(hipStreamSynchronize(c->stream));
    }
    return PW_OK;
}

uint64_t splitmix_next(uint64_t& s) {
    uint64_t z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

pw_status made_logq_host(pw_ctx c, const uint64_t* xs, int64_t count, double* logq) {
    auto& M = c->made;
    for (int64_t i = 0; i < count; i += M.maxB) {
        const int nb = (int)((count - i) < M.maxB ? (count - i) : M.maxB);
        pw_status s = made_stage(c, xs + i, nullptr, nb);
        if (s != PW_OK) return s;
        PW_HIP(made_forward(M.D, M.P, M.xs, nullptr, nb, nullptr, nullptr, nullptr, M.logq, c->stream));
        PW_HIP(hipMemcpyAsync(logq + i, M.logq, (size_t)nb * sizeof(double), hipMemcpyDeviceToHost, c->stream));
        PW_HIP(hipStreamSynchronize(c->stream));
    }
    return PW_OK;
}

}  // namespace

pw_status pw_made_param_count(int n, int hidden, size_t* count) {
    if (!count) return fail(PW_ERR_ARG, "null output");
    if (n < 2 || n > 32) return fail(PW_ERR_RANGE, "n=%d outside [2, 32]", n);
    if (hidden != 64 && hidden != 128 && hidden != 256) return fail(PW_ERR_UNSUPPORTED, "hidden must be 64, 128 or 256");
    *count = made_dims(n, hidden).total;
    return PW_OK;
}

pw_status pw_made_init(pw_ctx c, int n, int hidden, const double* params) {
    pw_status s = check_ctx(c);
    if (s != PW_OK) return s;
    size_t count = 0;
    s = pw_made_param_count(n, hidden, &count);
    if (s != PW_OK) return s;
    if (!params) return fail(PW_ERR_ARG, "null parameters");
    auto& M = c->made;
    if (M.block) {
        PW_HIP(hipStreamSynchronize(c->stream));
        PW_HIP(hipFree(M.block));
        M.block = nullptr;
    }
    M.ready = false;
    M.D = made_dims(n, hidden);
    M.maxB = MADE_MAXB;
    const size_t act = (size_t)M.maxB * hidden * sizeof(float);
    const size_t outb = (size_t)M.maxB * n * sizeof(float);
    size_t off = 0;
    auto carve = [&](size_t bytes) { size_t o = off; off += align256(bytes); return o; };
    const size_t oP = carve(count * 4), og = carve(count * 4), om = carve(count * 4), ov = carve(count * 4);
    const size_t oH1 = carve(act), oH2 = carve(act), oG1 = carve(act), oG2 = carve(act);
    const size_t oO = carve(outb), odO = carve(outb);
    const size_t olq = carve((size_t)M.maxB * 8), oxs = carve((size_t)M.maxB * 8), ow = carve((size_t)M.maxB * 4),
                 operm = carve((size_t)M.maxB * 4);
    if (fault(c, FAULT_ALLOC)) return fail(PW_ERR_HIP, "hipMalloc: injected failure");
    PW_HIP(hipMalloc(&M.block, off));
    char* b = (char*)M.block;
    M.P = (float*)(b + oP);
    M.g = (float*)(b + og);
    M.m = (float*)(b + om);
    M.v = (float*)(b + ov);
    M.H1 = (float*)(b + oH1);
    M.H2 = (float*)(b + oH2);
    M.G1 = (float*)(b + oG1);
    M.G2 = (float*)(b + oG2);
    M.O = (float*)(b + oO);
    M.dO = (float*)(b + odO);
    M.logq = (double*)(b + olq);
    M.xs = (uint64_t*)(b + oxs);
    M.w = (float*)(b + ow);
    M.perm = (int*)(b + operm);
    std::vector<float> pf(count);
    for (size_t i = 0; i < count; ++i) pf[i] = (float)params[i];
    PW_HIP(hipMemcpyAsync(M.P, pf.data(), count * 4, hipMemcpyHostToDevice, c->stream));
    PW_HIP(hipMemsetAsync(M.m, 0, count * 4, c->stream));
    PW_HIP(hipMemsetAsync(M.v, 0, count * 4, c->stream));
    PW_HIP(hipStreamSynchronize(c->stream));
    M.t = 0;
    M.ready = true;
    return PW_OK;
}

pw_status pw_made_get(pw_ctx c, double* params) {
    pw_status s = made_check(c);
    if (s != PW_OK) return s;
    if (!params) return fail(PW_ERR_ARG, "null output");
    std::vector<float> pf(c->made.D.total);
    PW_HIP(hipMemcpyAsync(pf.data(), c->made.P, pf.size() * 4, hipMemcpyDeviceToHost, c->stream));
    PW_HIP(hipStreamSynchronize(c->stream));
    for (size_t i = 0; i < pf.size(); ++i) params[i] = pf[i];
    return PW_OK;
}

pw_status pw_made_logq(pw_ctx c, const uint64_t* xs, int64_t count, double* logq) {
    pw_status s = made_check(c);
    if (s != PW_OK) return s;
    if (count < 0 || (count > 0 && (!xs || !logq))) return fail(PW_ERR_ARG, "bad arrays");
    for (int64_t i = 0; i < count; ++i)
        if (xs[i] >> c->made.D.n) return fail(PW_ERR_RANGE, "xs[%lld] has bits above n", (long long)i);
    return made_logq_host(c, xs, count, logq);
}

pw_status pw_made_grad(pw_ctx c, const uint64_t* xs, const double* w, int64_t count, double* loss, double* grad) {
    pw_status s = made_check(c);
    if (s != PW_OK) return s;
    auto& M = c->made;
    if (count < 1 || count > M.maxB) return fail(PW_ERR_RANGE, "count must be in [1, %d]", M.maxB);
    if (!xs || !w || !grad) return fail(PW_ERR_ARG, "null array");
    double W = 0.0;
    for (int64_t i = 0; i < count; ++i) {
        if (xs[i] >> M.D.n) return fail(PW_ERR_RANGE, "xs[%lld] has bits above n", (long long)i);
        if (!(w[i] >= 0.0)) return fail(PW_ERR_ARG, "weights must be >= 0");
        W += w[i];
    }
    if (!(W > 0.0)) return fail(PW_ERR_ARG, "weights sum to 0");
    s = made_stage(c, xs, w, count);
    if (s != PW_OK) return s;
    const int nb = (int)count;
    PW_HIP(made_forward(M.D, M.P, M.xs, nullptr, nb, M.H1, M.H2, M.O, M.logq, c->stream));
    PW_HIP(made_backward(M.D, M.P, M.xs, nullptr, M.w, (float)(1.0 / W), nb, M.H1, M.H2, M.O, M.dO, M.G1, M.G2,
                         c->stream));
    PW_HIP(made_wgrad(M.D, M.xs, nullptr, nb, M.dO, M.G1, M.G2, M.H1, M.H2, M.g, c->stream));
    std::vector<float> gf(M.D.total);
    std::vector<double> lq((size_t)count);
    PW_HIP(hipMemcpyAsync(gf.data(), M.g, gf.size() * 4, hipMemcpyDeviceToHost, c->stream));
    PW_HIP(hipMemcpyAsync(lq.data(), M.logq, lq.size() * 8, hipMemcpyDeviceToHost, c->stream));
    PW_HIP(hipStreamSynchronize(c->stream));
    for (size_t i = 0; i < gf.size(); ++i) grad[i] = gf[i];
    if (loss) {
        double l = 0.0;
        for (int64_t i = 0; i < count; ++i) l -= w[i] * lq[i];
        *loss = l / W;
    }
    return PW_OK;
}

pw_status pw_made_train(pw_ctx c, const uint64_t* xs, const double* w, int64_t count, int epochs, int minibatch,
                        double lr, uint64_t seed, double* final_loss) {
    pw_status s = made_check(c);
    if (s != PW_OK) return s;
    auto& M = c->made;
    if (count < 1) return fail(PW_ERR_ARG, "no training samples");
    if (minibatch < 1 || minibatch > M.maxB) return fail(PW_ERR_RANGE, "minibatch must be in [1, %d]", M.maxB);
    if (epochs < 0 || !(lr > 0.0)) return fail(PW_ERR_ARG, "bad epochs or learning rate");
    if (!xs || !w) return fail(PW_ERR_ARG, "null array");
    for (int64_t i = 0; i < count; ++i) {
        if (xs[i] >> M.D.n) return fail(PW_ERR_RANGE, "xs[%lld] has bits above n", (long long)i);
        if (!(w[i] >= 0.0)) return fail(PW_ERR_ARG, "weights must be >= 0");
    }
    std::vector<int64_t> order((size_t)count);
    std::vector<uint64_t> bx((size_t)minibatch);
    std::vector<double> bw((size_t)minibatch);
    for (int e = 0; e < epochs; ++e) {
        for (int64_t i = 0; i < count; ++i) order[i] = i;
        uint64_t st = seed ^ (0xA0761D6478BD642Full * (uint64_t)(e + 1));
        for (int64_t i = count - 1; i > 0; --i) {      // Fisher-Yates with SplitMix64
            const int64_t j = (int64_t)(splitmix_next(st) % (uint64_t)(i + 1));
            const int64_t t = order[i];
            order[i] = order[j];
            order[j] = t;
        }
        for (int64_t b0 = 0; b0 < count; b0 += minibatch) {
            const int nb = (int)((count - b0) < minibatch ? (count - b0) : minibatch);
            double W = 0.0;
            for (int i = 0; i < nb; ++i) {
                bx[i] = xs[order[b0 + i]];
                bw[i] = w[order[b0 + i]];
                W += bw[i];
            }
            if (!(W > 0.0)) continue;
            s = made_stage(c, bx.data(), bw.data(), nb);
            if (s != PW_OK) return s;
            PW_HIP(made_forward(M.D, M.P, M.xs, nullptr, nb, M.H1, M.H2, M.O, nullptr, c->stream));
            PW_HIP(made_backward(M.D, M.P, M.xs, nullptr, M.w, (float)(1.0 / W), nb, M.H1, M.H2, M.O, M.dO, M.G1,
                                 M.G2, c->stream));
            PW_HIP(made_wgrad(M.D, M.xs, nullptr, nb, M.dO, M.G1, M.G2, M.H1, M.H2, M.g, c->stream));
            ++M.t;
            PW_HIP(made_adam(M.P, M.g, M.m, M.v, M.D.total, (float)lr, 0.9f, 0.999f, 1e-8f, M.t, c->stream));
        }
    }
    PW_HIP(hipStreamSynchronize(c->stream));
    if (final_loss) {
        std::vector<double> lq((size_t)count);
        s = made_logq_host(c, xs, count, lq.data());
        if (s != PW_OK) return s;
        double l = 0.0, W = 0.0;
        for (int64_t i = 0; i < count; ++i) {
            l -= w[i] * lq[i];
            W += w[i];
        }
        *final_loss = l / W;
    }
    return PW_OK;
}

pw_status pw_made_sample(pw_ctx c, uint64_t seed, uint64_t offset, int64_t count, uint64_t* xs_out) {
    pw_status s = made_check(c);
    if (s != PW_OK) return s;
    if (count < 0 || (count > 0 && !xs_out)) return fail(PW_ERR_ARG, "bad output");
    auto& M = c->made;
    for (int64_t i = 0; i < count; i += M.maxB) {
        const int64_t nb = (count - i) < M.maxB ? (count - i) : M.maxB;
        PW_HIP(made_sample(M.D, M.P, seed, offset + (uint64_t)i, nb, M.xs, c->stream));
        PW_HIP(hipMemcpyAsync(xs_out + i, M.xs, (size_t)nb * 8, hipMemcpyDeviceToHost, c->stream));
        PW_HIP(hipStreamSynchronize(c->stream));
    }
    return PW_OK;
}

namespace {
// Monte Carlo with the learned proposal (see pw_mc_learned).  mode: 0 = defensive mixture
// with the defensive component chosen from the pilot; 1 = the same, but when a held-out
// quarter of the pilot predicts that plain sampling (uniform or marginal) spreads less
// than the mixture, that sampler runs instead.  *chosen: 0 uniform, 1 marginal, 2 mixture
// with the uniform, 3 mixture with the marginal; pred[3]: predicted r_2 of uniform,
// marginal and mixture (held-out quarter; NaN where not computed).
pw_status mc_learned_core(pw_ctx c, double eps, int batch, uint64_t max_samples, double target_se, uint64_t seed,
                          double lambda, int64_t pilot, int epochs, int minibatch, double lr, int mode, int* chosen,
                          double* pred, pw_result* out) {
    pw_status s = check_state(c);
    if (s != PW_OK) return s;
    s = made_check(c);
    if (s != PW_OK) return s;
    if (!out) return fail(PW_ERR_ARG, "null output");
    if (c->made.D.n != c->n) return fail(PW_ERR_ARG, "learned proposal has n=%d, state has n=%d", c->made.D.n, c->n);
    if (!(lambda > 0.0 && lambda <= 1.0)) return fail(PW_ERR_ARG, "lambda must be in (0, 1]");
    if (batch < 1 || batch > c->made.maxB) return fail(PW_ERR_ARG, "batch must be in [1, %d]", c->made.maxB);
    if (pilot < 8 || max_samples < 3) return fail(PW_ERR_ARG, "need pilot >= 8 and max_samples >= 3");
    if (!(eps >= 0.0 && eps < 1.0)) return fail(PW_ERR_ARG, "eps=%g outside [0, 1)", eps);
    const int n = c->n;
    const double d = ldexp(1.0, n);
    FamilyRes r0;
    const uint64_t zero = 0;
    s = eval_host(c, &zero, 1, eps, &r0);
    if (s != PW_OK) return s;
    const double p0 = r0.p;
    if (!(p0 < 1.0 - 1e-12)) return fail(PW_ERR_UNSUPPORTED, "p(0) = %.17g: no mass on x != 0", p0);
    // pilot: x ~ p(. | x != 0), training targets t(x) ~ m_2(x), i.e. weights m_2(x) / p(x)
    std::vector<uint64_t> px((size_t)pilot);
    std::vector<FamilyRes> pr((size_t)pilot);
    s = pw_sample_x(c, PW_SAMPLER_MARGINAL_NZ, seed, 0, pilot, px.data());
    if (s != PW_OK) return s;
    for (int64_t i = 0; i < pilot; ++i)
        if (px[i] == 0) return fail(PW_ERR_UNSUPPORTED, "the marginal sampler drew x = 0 (|psi|^2 is a point mass)");
    s = eval_host(c, px.data(), pilot, eps, pr.data());
    if (s != PW_OK) return s;
    // the defensive component: the plain sampler with the smaller spread on the pilot
    std::vector<DrawMP> dm((size_t)pilot);
    for (int64_t i = 0; i < pilot; ++i) dm[(size_t)i] = {pr[i].m[0], pr[i].p};
    const Spreads sp = spreads_from_marginal_pilot(dm, r0.m[0], p0, d);
    const bool def_uniform = sp.r_uniform < sp.r_marginal;
    // train on the first three quarters (all of the pilot in mode 0)
    const int64_t ntrain = mode == 1 ? pilot - pilot / 4 : pilot;
    std::vector<double> pw_((size_t)ntrain);
    for (int64_t i = 0; i < ntrain; ++i) pw_[i] = pr[i].m[0] / pr[i].p;
    s = pw_made_train(c, px.data(), pw_.data(), ntrain, epochs, minibatch, lr, seed ^ 0x5EEDull, nullptr);
    if (s != PW_OK) return s;
    double lq0 = 0.0;
    s = made_logq_host(c, &zero, 1, &lq0);
    if (s != PW_OK) return s;
    const double q0 = exp(lq0);
    // proposal density on x != 0 of the mixture
    auto qmix = [&](double p, double lqx) {
        const double qd = def_uniform ? 1.0 / (d - 1.0) : p / (1.0 - p0);
        return lambda * qd + (1.0 - lambda) * exp(lqx) / (1.0 - q0);
    };
    int pick = def_uniform ? 2 : 3;
    double pr3[3] = {NAN, NAN, NAN};
    if (mode == 1) {
        // held-out quarter, x ~ p_c = p / (1 - p0): the second moment of m / g under a
        // proposal g is E_{p_c}[m^2 / (g p_c)]; its mean is S - m_0 for every g
        const int64_t h0 = ntrain, nh = pilot - ntrain;
        std::vector<double> lqh((size_t)nh);
        s = made_logq_host(c, px.data() + h0, nh, lqh.data());
        if (s != PW_OK) return s;
        double mu = 0.0, su = 0.0, sm = 0.0, sx = 0.0;
        for (int64_t i = 0; i < nh; ++i) {
            const double m = pr[h0 + i].m[0], p = pr[h0 + i].p, pc = p / (1.0 - p0);
            mu += m / pc;
            su += m * m * (d - 1.0) / pc;           // g = 1 / (d - 1)
            sm += m * m / (pc * pc);                // g = p_c
            sx += m * m / (qmix(p, lqh[i]) * pc);   // g = the mixture
        }
        mu /= (double)nh;
        const double S = r0.m[0] + mu;
        auto rr = [&](double second) { return sqrt(fmax(second / (double)nh - mu * mu, 0.0)) / S; };
        pr3[0] = rr(su);
        pr3[1] = rr(sm);
        pr3[2] = rr(sx);
        if (pr3[0] < pr3[2] || pr3[1] < pr3[2]) pick = pr3[0] < pr3[1] ? 0 : 1;
    }
    if (chosen) *chosen = pick;
    if (pred)
        for (int k = 0; k < 3; ++k) pred[k] = pr3[k];
    if (pick < 2) {
        // plain sampling judged better: the estimator of pw_mc on a stream of its own
        return pw_mc(c, pick == 0 ? PW_SAMPLER_UNIFORM_NZ : PW_SAMPLER_MARGINAL_NZ, eps, batch, max_samples,
                     target_se, seed + 0x9E3779B97F4A7C15ull, out);
    }
    // defensive mixture q = lambda q_def + (1 - lambda) q_theta(.|x != 0), exact weights m / q
    Running run[4];
    double gap = r0.gap;
    uint64_t drawn = 0;
    const uint64_t draws_max = max_samples - 1;
    std::vector<uint64_t> xm, xl, xs;
    std::vector<FamilyRes> res;
    std::vector<double> lq;
    int batches = 0;
    const uint64_t seed_mc = seed + 0x9E3779B97F4A7C15ull;
    while (drawn < draws_max) {
        const int64_t nb = (int64_t)((draws_max - drawn) < (uint64_t)batch ? (draws_max - drawn) : (uint64_t)batch);
        xm.resize((size_t)nb);
        xl.resize((size_t)nb);
        xs.resize((size_t)nb);
        res.resize((size_t)nb);
        lq.resize((size_t)nb);
        s = pw_sample_x(c, def_uniform ? PW_SAMPLER_UNIFORM_NZ : PW_SAMPLER_MARGINAL_NZ, seed_mc, drawn, nb, xm.data());
        if (s != PW_OK) return s;
        s = pw_made_sample(c, seed_mc, drawn, nb, xl.data());
        if (s != PW_OK) return s;
        for (int64_t i = 0; i < nb; ++i) {
            uint64_t W0, W1;
            philox_words(seed_mc, drawn + (uint64_t)i, 0u, STREAM_MIX, W0, W1);
            const double u = (double)(W0 >> 11) * 0x1.0p-53;
            xs[i] = u < lambda ? xm[i] : xl[i];
            if (xs[i] == 0) return fail(PW_ERR_UNSUPPORTED, "a sampler could not draw x != 0 in 64 attempts");
        }
        s = eval_host(c, xs.data(), nb, eps, res.data());
        if (s != PW_OK) return s;
        s = made_logq_host(c, xs.data(), nb, lq.data());
        if (s != PW_OK) return s;
        for (int64_t i = 0; i < nb; ++i) {
            const FamilyRes& f = res[i];
            const double wgt = 1.0 / qmix(f.p, lq[i]);
            for (int a = 0; a < 3; ++a) run[a].add(wgt * f.m[a]);
            run[3].add(wgt * f.ent);
            gap = fmax(gap, f.gap);
        }
        drawn += (uint64_t)nb;
        ++batches;
        const double S2 = r0.m[0] + run[0].mean;
        const double Mse = sqrt(run[0].var() / run[0].n) / (log(2.0) * S2);
        if (batches >= 2 && target_se > 0 && Mse <= target_se) break;
    }
    pw_result r;
    memset(&r, 0, sizeof r);
    for (int a = 0; a < 3; ++a) {
        const double S = r0.m[a] + run[a].mean;
        const double se = sqrt(run[a].var() / run[a].n);
        r.S[a] = S;
        r.S_se[a] = se;
        r.M[a] = log2(S) / (1.0 - (a + 2)) - n;
        r.M_se[a] = se / (fabs(1.0 - (a + 2)) * log(2.0) * S);
        r.r[a] = sqrt(run[a].var()) / S;
    }
    r.L = r0.ent + run[3].mean;
    r.L_se = sqrt(run[3].var() / run[3].n);
    r.M1 = -r.L / d;
    r.M1_se = r.L_se / d;
    r.P = NAN;
    r.nullity = NAN;
    r.n_samples = drawn + 1;
    r.gap = gap;
    *out = r;
    return PW_OK;
}
}  // namespace

pw_status pw_mc_learned(pw_ctx c, double eps, int batch, uint64_t max_samples, double target_se, uint64_t seed,
                        double lambda, int64_t pilot, int epochs, int minibatch, double lr, pw_result* out) {
    return mc_learned_core(c, eps, batch, max_samples, target_se, seed, lambda, pilot, epochs, minibatch, lr, 0,
                           nullptr, nullptr, out);
}

pw_status pw_mc_learned_auto(pw_ctx c, double eps, int batch, uint64_t max_samples, double target_se, uint64_t seed,
                             double lambda, int64_t pilot, int epochs, int minibatch, double lr, int* chosen,
                             double* predicted_r2, pw_result* out) {
    return mc_learned_core(c, eps, batch, max_samples, target_se, seed, lambda, pilot, epochs, minibatch, lr, 1,
                           chosen, predicted_r2, out);
}

pw_status pw_mixed(pw_ctx c, int n_a, double eps, pw_mixed_result* out) {
    pw_status s = check_state(c);
    if (s != PW_OK) return s;
    if (!out) return fail(PW_ERR_ARG, "null output");
    const bool dbl = c->dtype == PW_C128;
    if (n_a < 1 || n_a > c->n || n_a > MIXED_MAX_QUBITS)
        return fail(PW_ERR_RANGE, "n_a=%d outside [1, min(n, %d)]", n_a, MIXED_MAX_QUBITS);
    if (!(eps >= 0.0 && eps < 1.0)) return fail(PW_ERR_ARG, "eps=%g outside [0, 1)", eps);
    const size_t dA = (size_t)1 << n_a;
    // library-owned: the family-major rho_A, then (families larger than one workgroup
    // holds) the multi-pass work and partials for nbm families per launch
    const Plan P = make_plan(n_a, dbl);
    const size_t half_bytes = (dA >> 1) * esize(c->dtype);
    size_t nbm = MAX_BATCH, work_b = 0, parts_b = 0;
    if (!P.fused) {
        nbm = ((size_t)256 << 20) / half_bytes;
        nbm = nbm < 1 ? 1 : (nbm > 256 ? 256 : nbm);
        work_b = align256(nbm * half_bytes);
        parts_b = align256(nbm * (size_t)P.blocks_last * sizeof(FamilyRes));
    }
    const size_t rho_b = align256(dA * dA * esize(c->dtype));
    const size_t bytes = rho_b + work_b + parts_b;
    if (c->rho_bytes < bytes) {
        if (c->rho) {
            PW_HIP(hipStreamSynchronize(c->stream));
            PW_HIP(hipFree(c->rho));
            c->rho = nullptr;
            c->rho_bytes = 0;
        }
        if (fault(c, FAULT_ALLOC)) return fail(PW_ERR_HIP, "hipMalloc: injected failure");
        PW_HIP(hipMalloc(&c->rho, bytes));
        c->rho_bytes = bytes;
    }
    if (fault(c, FAULT_LAUNCH)) return fail(PW_ERR_HIP, "kernel launch: injected failure");
    PW_HIP(reduced_density(dbl, c->psi, c->n, n_a, c->rho, c->stream, timer_of(c)));
    FamilyRes* fam = at<FamilyRes>(c, c->L.fam);
    void* work = (char*)c->rho + rho_b;
    FamilyRes* parts = reinterpret_cast<FamilyRes*>((char*)c->rho + rho_b + work_b);
    for (size_t x0 = 0; x0 < dA; x0 += nbm) {
        const int nb = (int)((dA - x0) < nbm ? (dA - x0) : nbm);
        PW_HIP(eval_reduced_batch(dbl, c->max_alpha, c->rho, n_a, x0, nb, eps, work, parts, fam + x0, c->stream));
    }
    SweepSums* sw = at<SweepSums>(c, c->L.sweep);
    PW_HIP(reduce_families(fam, (int64_t)dA, sw, c->stream));
    PW_HIP(reduce_sweep(sw, reduce_families_slots((int64_t)dA), sw + SWEEP_SLOTS, c->stream));
    SweepSums h;
    PW_HIP(hipMemcpyAsync(&h, sw + SWEEP_SLOTS, sizeof h, hipMemcpyDeviceToHost, c->stream));
    PW_HIP(hipStreamSynchronize(c->stream));
    pw_mixed_result r;
    memset(&r, 0, sizeof r);
    r.purity = h.P;
    r.S2 = -log2(h.P);
    for (int a = 0; a < 3; ++a) {
        r.W[a] = h.S[a];
        r.M[a] = log2(h.S[a]) / (1.0 - (a + 2)) - n_a - r.S2;
    }
    r.L = h.L;
    r.families = h.count;
    *out = r;
    return PW_OK;
}

extern "C++" {
namespace {
// Candidate schedules of the bound state: the plan variants that apply (first pass of 12 or
// 15 bits, column tiles of 12 / 13 / 15 bits) crossed with the first-pass groups that the
// plan and the launch size allow.
std::vector<Schedule> schedule_candidates(pw_ctx c) {
    std::vector<Schedule> out;
    if (c->P.fused || c->cmfma) {
        out.push_back(Schedule{0, 0, 0});
        return out;
    }
    const int nh = c->n - 1;
    std::vector<std::pair<int, int>> plans;
    if (c->cdbl) {
        plans.push_back({12, 12});
    } else {
        plans.push_back({12, 12});
        plans.push_back({12, 13});
        const int sb = nh - 15;
        if (sb >= 1 && sb <= 12) {
            if (sb <= 8) plans.push_back({15, 12});
            if (sb <= 9) plans.push_back({15, 13});
            if (sb >= 9) plans.push_back({15, 15});
        }
    }
    for (auto& pk : plans) {
        bool ok = true;
        const Plan P = make_plan_sched(c->n, c->cdbl, Schedule{pk.first, pk.second, 1}, &ok);
        if (!ok) continue;
        const bool can_group = P.nh - P.k1 >= 3;
        for (int g = 1; g <= GROUP_MAX; g *= 2) {
            if (g > 1 && (!can_group || g > c->batch)) continue;
            out.push_back(Schedule{pk.first, pk.second, g});
        }
    }
    return out;
}
}  // namespace
}  // extern "C++"

pw_status pw_autotune(pw_ctx c, int* best_batch, int* candidates, double* us_per_family, int* n_candidates) {
    pw_status s = check_state(c);
    if (s != PW_OK) return s;
    if (!best_batch) return fail(PW_ERR_ARG, "null output");
    if (fault(c, FAULT_LAUNCH)) return fail(PW_ERR_HIP, "kernel launch: injected failure");
    s = ensure_compute_state(c);
    if (s != PW_OK) return s;
    // the timed work is what Monte Carlo steps and device lists run: a list of uniformly
    // drawn x (Philox stream keyed 0x7475) through the sorted, grouped evaluation
    const uint64_t d = 1ull << c->n;
    int64_t total = 4 * (int64_t)c->batch;
    if (total > c->L.xcap) total = c->L.xcap;
    if ((uint64_t)total > d - 1) total = (int64_t)(d - 1);
    if (total < 1) total = 1;
    uint64_t* dx = at<uint64_t>(c, c->L.xs);
    PW_HIP(sample_uniform(c->n, 0x7475, 0, total, dx, c->stream));
    hipEvent_t e0, e1;
    PW_HIP(hipEventCreate(&e0));
    PW_HIP(hipEventCreate(&e1));
    const Plan saved_P = c->P;
    const int saved = c->run_batch;
    const int saved_every = c->timing_every;
    c->timing_every = 0;
    FamilyRes* fam = at<FamilyRes>(c, c->L.fam);
    // microseconds per family of the current plan and launch size (best of two after a warm-up)
    auto time_it = [&](double* us) -> pw_status {
        double tmin = 1e300;
        for (int rep = 0; rep < 3; ++rep) {
            PW_HIP(hipEventRecord(e0, c->stream));
            const pw_status st = eval_device(c, dx, 0, total, 1e-4, fam);
            if (st != PW_OK) return st;
            PW_HIP(hipEventRecord(e1, c->stream));
            PW_HIP(hipEventSynchronize(e1));
            float ms = 0.f;
            PW_HIP(hipEventElapsedTime(&ms, e0, e1));
            if (rep > 0) tmin = fmin(tmin, (double)ms);
        }
        *us = 1e3 * tmin / (double)total;
        return PW_OK;
    };
    // stage 1: plan variant and group at the workspace's launch size
    Schedule best_sc{0, 0, 0};
    double best = 1e300;
    c->run_batch = c->batch;
    for (const Schedule& sc : schedule_candidates(c)) {
        bool ok = true;
        c->P = c->cmfma ? make_plan_bf16x2(c->n) : make_plan_sched(c->n, c->cdbl, sc, &ok);
        double us = 0.0;
        s = time_it(&us);
        if (s != PW_OK) break;
        if (us < best) {
            best = us;
            best_sc = sc;
        }
    }
    // stage 2: families per launch for that schedule (none below its group)
    std::vector<int> cand;
    std::vector<double> times;
    int bestb = c->batch;
    if (s == PW_OK) {
        bool ok = true;
        c->P = c->cmfma ? make_plan_bf16x2(c->n) : make_plan_sched(c->n, c->cdbl, best_sc, &ok);
        const int bmin = first_pass_group(c->P, c->cdbl, c->batch);
        for (int b = c->batch; b >= bmin && (int)cand.size() < 6; b /= 2) cand.push_back(b);
        if (cand.empty()) cand.push_back(c->batch);
        best = 1e300;
        for (int b : cand) {
            c->run_batch = b;
            double us = 0.0;
            s = time_it(&us);
            if (s != PW_OK) break;
            times.push_back(us);
            if (us < best) {
                best = us;
                bestb = b;
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    c->timing_every = saved_every;
    if (s != PW_OK) {
        c->P = saved_P;
        c->run_batch = saved;
        return s;
    }
    tuned_put(c->device, c->n, prec_key(c, c->dtype), Tuned{best_sc, bestb, best});
    // the tuned schedule takes effect unless the context asked for its own
    c->P = saved_P;
    apply_schedule(c, c->dtype);
    *best_batch = bestb;
    if (n_candidates) *n_candidates = (int)times.size();
    for (size_t i = 0; i < times.size(); ++i) {
        if (candidates) candidates[i] = cand[i];
        if (us_per_family) us_per_family[i] = times[i];
    }
    return PW_OK;
}

pw_status pw_set_schedule(pw_ctx c, int first_bits, int column_tile_bits, int group, int batch) {
    pw_status s = check_ctx(c);
    if (s != PW_OK) return s;
    if ((first_bits != 0 && first_bits != 12 && first_bits != 15) ||
        (column_tile_bits != 0 && column_tile_bits != 12 && column_tile_bits != 13 && column_tile_bits != 15) ||
        group < 0 || group > GROUP_MAX || (group & (group - 1)) != 0 || batch < 0 ||
        batch > MAX_BATCH)
        return fail(PW_ERR_ARG, "schedule (%d, %d, %d, %d) outside the supported values", first_bits,
                    column_tile_bits, group, batch);
    const Schedule sc{first_bits, column_tile_bits, group};
    if (c->bound && !c->cmfma) {
        bool ok = true;
        (void)make_plan_sched(c->n, c->cdbl, sc, &ok);
        if (!ok)
            return fail(PW_ERR_UNSUPPORTED, "schedule (%d, %d, %d) does not apply to n=%d", first_bits,
                        column_tile_bits, group, c->n);
    }
    c->sched = sc;
    c->sched_batch = batch;
    if (c->bound) apply_schedule(c, c->dtype);
    return PW_OK;
}

pw_status pw_get_schedule(pw_ctx c, int* first_bits, int* column_tile_bits, int* group, int* batch) {
    pw_status s = check_state(c);
    if (s != PW_OK) return s;
    if (first_bits) *first_bits = c->P.fused ? 0 : c->P.k1;
    if (column_tile_bits) *column_tile_bits = c->P.fused ? 0 : c->P.ktile;
    if (group) *group = first_pass_group(c->P, c->cdbl, c->run_batch);
    if (batch) *batch = c->run_batch;
    return PW_OK;
}

pw_status pw_autotune_save(const char* path) {
    if (!path) return fail(PW_ERR_ARG, "null path");
    FILE* f = fopen(path, "w");
    if (!f) return fail(PW_ERR_ARG, "cannot write %s", path);
    std::lock_guard<std::mutex> lk(g_tune_mu);
    fprintf(f, "# pauliwht autotune v1: device-name n arithmetic first_bits column_tile_bits group batch us_per_family\n");
    for (const auto& kv : g_tune) {
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, std::get<0>(kv.first)) != hipSuccess) continue;
        const Tuned& t = kv.second;
        fprintf(f, "%s %d %d %d %d %d %d %.6g\n", prop.gcnArchName, std::get<1>(kv.first), std::get<2>(kv.first),
                t.sc.first_bits, t.sc.column_tile_bits, t.sc.group, t.batch, t.us);
    }
    fclose(f);
    return PW_OK;
}

pw_status pw_autotune_load(const char* path, int* loaded) {
    if (!path) return fail(PW_ERR_ARG, "null path");
    FILE* f = fopen(path, "r");
    if (!f) return fail(PW_ERR_ARG, "cannot read %s", path);
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess) ndev = 0;
    std::vector<std::string> names;
    for (int i = 0; i < ndev; ++i) {
        hipDeviceProp_t prop;
        names.push_back(hipGetDeviceProperties(&prop, i) == hipSuccess ? std::string(prop.gcnArchName) : "");
    }
    char line[512];
    int cnt = 0;
    while (fgets(line, sizeof line, f)) {
        if (line[0] == '#') continue;
        char name[256];
        int n, key, fb, ct, g, b;
        double us;
        if (sscanf(line, "%255s %d %d %d %d %d %d %lf", name, &n, &key, &fb, &ct, &g, &b, &us) != 8) continue;
        if (n < 1 || n > MAX_QUBITS || key < 0 || key > 2 || b < 0 || b > MAX_BATCH) continue;
        for (int i = 0; i < ndev; ++i)
            if (names[(size_t)i] == name) {
                tuned_put(i, n, key, Tuned{Schedule{fb, ct, g}, b, us});
                ++cnt;
            }
    }
    fclose(f);
    if (loaded) *loaded = cnt;
    return PW_OK;
}

pw_status pw_eval_states(pw_ctx c, int nstates, const pw_state_ref* states, const int* state_idx,
                         const uint64_t* xs, int64_t n_x, double eps, pw_xres* out) {
    pw_status s = check_ctx(c);
    if (s != PW_OK) return s;
    if (nstates < 1 || !states) return fail(PW_ERR_ARG, "no states");
    if (n_x < 0 || (n_x > 0 && (!state_idx || !xs || !out))) return fail(PW_ERR_ARG, "bad arrays");
    if (!(eps >= 0.0 && eps < 1.0)) return fail(PW_ERR_ARG, "eps=%g outside [0, 1)", eps);
    for (int k = 0; k < nstates; ++k) {
        const pw_state_ref& r = states[k];
        if (!r.psi || ((uintptr_t)r.psi & 255)) return fail(PW_ERR_ARG, "state %d: null or unaligned pointer", k);
        if (r.dtype != PW_C128 && r.dtype != PW_C64) return fail(PW_ERR_ARG, "state %d: unknown dtype", k);
        if (r.n < 1 || r.n > MAX_QUBITS) return fail(PW_ERR_RANGE, "state %d: n=%d outside [1, %d]", k, r.n, MAX_QUBITS);
    }
    for (int64_t i = 0; i < n_x; ++i) {
        if (state_idx[i] < 0 || state_idx[i] >= nstates) return fail(PW_ERR_ARG, "state_idx[%lld] out of range", (long long)i);
        if (xs[i] >> states[state_idx[i]].n) return fail(PW_ERR_RANGE, "xs[%lld] not below 2^n of its state", (long long)i);
    }
    // one workspace shared by all states; each state runs at its own families-per-launch
    // (its default, shrunk to fit a caller-owned workspace), and the workspace holds the
    // largest of those layouts
    std::vector<int> Bk((size_t)nstates);
    size_t need = 0;
    for (int k = 0; k < nstates; ++k) {
        int b = default_batch(states[k].n, states[k].dtype);
        if (c->ws && !c->ws_owned)
            while (b > 1 && layout_for(states[k].n, states[k].dtype, b).total > c->ws_bytes) b /= 2;
        Bk[(size_t)k] = b;
        need = std::max(need, layout_for(states[k].n, states[k].dtype, b).total);
    }
    if (c->ws && !c->ws_owned && need > c->ws_bytes)
        return fail(PW_ERR_WORKSPACE, "workspace too small for the largest state");
    const bool was_bound = c->bound;
    void* const saved_psi = c->psi;
    const int saved_n = c->n;
    const pw_dtype saved_dt = c->dtype;
    // puts the caller's bound state back (the workspace stays carved for the largest
    // state); every exit from here on goes through it, so a failed call also keeps it
    auto restore = [&](pw_status st) -> pw_status {
        c->psi = saved_psi;
        c->n = saved_n;
        c->dtype = saved_dt;
        c->bound = false;
        c->cdf_valid = false;
        if (was_bound) {
            const pw_status s2 = prepare_workspace(c, saved_n, saved_dt);
            if (s2 == PW_OK) c->bound = true;
            if (st == PW_OK) st = s2;
        }
        return st;
    };
    // the list grouped by state (a stable counting sort; positions kept for the scatter)
    std::vector<int64_t> start((size_t)nstates + 1, 0), order((size_t)n_x);
    for (int64_t i = 0; i < n_x; ++i) ++start[(size_t)state_idx[i] + 1];
    for (int k = 0; k < nstates; ++k) start[(size_t)k + 1] += start[(size_t)k];
    {
        std::vector<int64_t> fill(start.begin(), start.end() - 1);
        for (int64_t i = 0; i < n_x; ++i) order[(size_t)fill[(size_t)state_idx[i]]++] = i;
    }
    // classes of states with the same n and dtype, each evaluated as one list whose
    // launches span its states; inside a class the families go state by state, each
    // state's in top-bit order (x = 0 first), so that the first pass's tile-sharing groups
    // meet families of one state and one top bit
    std::vector<int> cls_of((size_t)nstates, -1);
    std::vector<std::vector<int>> classes;
    for (int k = 0; k < nstates; ++k) {
        if (start[(size_t)k + 1] == start[(size_t)k]) continue;
        for (size_t q = 0; q < classes.size() && cls_of[(size_t)k] < 0; ++q) {
            const int r = classes[q][0];
            if (states[r].n == states[k].n && states[r].dtype == states[k].dtype) {
                classes[q].push_back(k);
                cls_of[(size_t)k] = (int)q;
            }
        }
        if (cls_of[(size_t)k] < 0) {
            cls_of[(size_t)k] = (int)classes.size();
            classes.push_back({k});
        }
    }
    std::vector<int64_t> seq;   // positions in evaluation order
    std::vector<int64_t> cstart(classes.size() + 1, 0);
    seq.reserve((size_t)n_x);
    for (size_t q = 0; q < classes.size(); ++q) {
        cstart[q] = (int64_t)seq.size();
        for (int k : classes[q]) {
            int64_t cnt[34] = {0};
            auto key = [&](int64_t pos) { const uint64_t x = xs[pos]; return x ? 64 - __builtin_clzll(x) : 0; };
            for (int64_t j = start[(size_t)k]; j < start[(size_t)k + 1]; ++j) ++cnt[key(order[(size_t)j]) + 1];
            for (int b = 0; b < 33; ++b) cnt[b + 1] += cnt[b];
            const size_t base = seq.size();
            seq.resize(base + (size_t)(start[(size_t)k + 1] - start[(size_t)k]));
            for (int64_t j = start[(size_t)k]; j < start[(size_t)k + 1]; ++j) {
                const int64_t pos = order[(size_t)j];
                seq[base + (size_t)cnt[key(pos)]++] = pos;
            }
        }
    }
    cstart[classes.size()] = (int64_t)seq.size();
    // pinned host staging (norms, grouped x, results) and the states' norm slots on the
    // device: the whole call synchronises twice, once for the norm checks of all states
    // and once for all results
    const size_t o_x = align256((size_t)nstates * 2 * sizeof(double));
    const size_t o_p = o_x + align256((size_t)n_x * sizeof(uint64_t));
    const size_t o_r = o_p + align256((size_t)n_x * sizeof(uint64_t));
    const size_t pin_need = o_r + align256((size_t)n_x * sizeof(FamilyRes));
    const size_t nrm_need = (size_t)nstates * 2 * sizeof(double);
    auto allocate = [&]() -> pw_status {
        if (!(c->ws && !c->ws_owned) && (!c->ws || c->ws_bytes < need)) {
            c->cdf_valid = false;  // the bound state's tables do not survive this
            if (c->ws) {
                PW_HIP(hipStreamSynchronize(c->stream));
                PW_HIP(hipFree(c->ws));
                c->ws = nullptr;
                c->ws_bytes = 0;
            }
            if (fault(c, FAULT_ALLOC)) return fail(PW_ERR_HIP, "hipMalloc: injected failure");
            void* p = nullptr;
            PW_HIP(hipMalloc(&p, need));
            c->ws = (char*)p;
            c->ws_bytes = need;
            c->ws_owned = true;
        }
        if (c->pin_bytes < pin_need) {
            if (c->pin) {
                PW_HIP(hipStreamSynchronize(c->stream));
                PW_HIP(hipHostFree(c->pin));
                c->pin = nullptr;
                c->pin_bytes = 0;
            }
            if (fault(c, FAULT_ALLOC)) return fail(PW_ERR_HIP, "hipHostMalloc: injected failure");
            PW_HIP(hipHostMalloc(&c->pin, pin_need, hipHostMallocDefault));
            c->pin_bytes = pin_need;
        }
        if (c->nrm_bytes < nrm_need) {
            if (c->nrm) {
                PW_HIP(hipStreamSynchronize(c->stream));
                PW_HIP(hipFree(c->nrm));
                c->nrm = nullptr;
                c->nrm_bytes = 0;
            }
            if (fault(c, FAULT_ALLOC)) return fail(PW_ERR_HIP, "hipMalloc: injected failure");
            PW_HIP(hipMalloc(&c->nrm, nrm_need));
            c->nrm_bytes = nrm_need;
        }
        return PW_OK;
    };
    s = allocate();
    if (s != PW_OK) return restore(s);
    const size_t cap = c->ws_bytes;
    double* hnorm = reinterpret_cast<double*>(c->pin);
    uint64_t* hx = reinterpret_cast<uint64_t*>((char*)c->pin + o_x);
    uint64_t* hp = reinterpret_cast<uint64_t*>((char*)c->pin + o_p);
    FamilyRes* hres = reinterpret_cast<FamilyRes*>((char*)c->pin + o_r);
    for (int64_t j = 0; j < n_x; ++j) {
        hx[j] = xs[seq[(size_t)j]];
        hp[j] = (uint64_t)(uintptr_t)states[state_idx[seq[(size_t)j]]].psi;
    }
    double* dnrm = reinterpret_cast<double*>(c->nrm);
    // bind state k's plan and layout to the context
    auto use_state = [&](int k) -> pw_status {
        c->psi = states[k].psi;
        c->n = states[k].n;
        c->dtype = states[k].dtype;
        // each state in its own storage precision (complex64 states take the split-BF16
        // transform when the context asks for it)
        c->cdbl = c->dtype == PW_C128;
        c->cmfma = !c->cdbl && c->prec == PW_PREC_BF16X2;
        c->cpsi = c->psi;
        c->conv_valid = true;
        const int B = Bk[(size_t)k];
        c->L = layout_for(c->n, c->dtype, B);
        if (c->L.total > cap) return fail(PW_ERR_WORKSPACE, "state %d does not fit the shared workspace", k);
        c->batch = B;
        Tuned t{};
        const bool have = tuned_get(c->device, c->n, c->cdbl ? 0 : c->cmfma ? 2 : 1, &t);
        bool ok = true;
        c->P = c->cmfma ? make_plan_bf16x2(c->n) : make_plan_sched(c->n, c->cdbl, have ? t.sc : Schedule{0, 0, 0}, &ok);
        c->run_batch = have && t.batch > 0 && t.batch < B ? t.batch : B;
        c->cdf_valid = false;
        return PW_OK;
    };
    // 1. the norm of every state that has families (stream order keeps the shared
    //    partial-sum region of one state from being overwritten before it is reduced)
    for (int k = 0; k < nstates && s == PW_OK; ++k) {
        if (start[(size_t)k + 1] == start[(size_t)k]) continue;
        s = use_state(k);
        if (s != PW_OK) break;
        unsigned* bad = reinterpret_cast<unsigned*>(dnrm + 2 * k + 1);
        if (hipMemsetAsync(bad, 0, sizeof(unsigned), c->stream) != hipSuccess ||
            norm2(c->dtype == PW_C128, c->psi, c->n, at<double>(c, c->L.norm), norm2_parts(c->n), dnrm + 2 * k, bad,
                  c->stream) != hipSuccess)
            s = fail(PW_ERR_HIP, "state %d: norm launch failed", k);
    }
    if (s == PW_OK) {
        if (hipMemcpyAsync(hnorm, dnrm, nrm_need, hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
            hipStreamSynchronize(c->stream) != hipSuccess)
            s = fail(PW_ERR_HIP, "norm copy failed");
    }
    for (int k = 0; k < nstates && s == PW_OK; ++k) {
        if (start[(size_t)k + 1] == start[(size_t)k]) continue;
        unsigned hb;
        memcpy(&hb, hnorm + 2 * k + 1, sizeof hb);
        const double nrm = hnorm[2 * k];
        const double tol = states[k].dtype == PW_C128 ? 1e-10 : 1e-5;
        if (hb) s = fail(PW_ERR_NOT_NORMALIZED, "state %d holds NaN or Inf amplitudes", k);
        else if (!(fabs(nrm - 1.0) <= tol)) s = fail(PW_ERR_NOT_NORMALIZED, "state %d: <psi|psi> = %.17g", k, nrm);
    }
    // 2. each class's families as one list (x and state address in, results out through
    //    the pinned staging), no synchronisation until the end (each copy and launch is
    //    ordered on the stream); the state addresses take the sorted-list staging, which a
    //    list in this order does not need
    for (size_t q = 0; q < classes.size() && s == PW_OK; ++q) {
        const int64_t j0 = cstart[q], j1 = cstart[q + 1];
        s = use_state(classes[q][0]);
        if (s != PW_OK) break;
        if (fault(c, FAULT_LAUNCH)) {
            s = fail(PW_ERR_HIP, "kernel launch: injected failure");
            break;
        }
        s = ensure_compute_state(c);
        if (s != PW_OK) break;
        uint64_t* dx = at<uint64_t>(c, c->L.xs);
        uint64_t* dp = at<uint64_t>(c, c->L.xsort);
        FamilyRes* dr = at<FamilyRes>(c, c->L.xres);
        for (int64_t j = j0; j < j1 && s == PW_OK; j += c->L.xcap) {
            const int64_t nb = (j1 - j) < c->L.xcap ? (j1 - j) : c->L.xcap;
            if (hipMemcpyAsync(dx, hx + j, (size_t)nb * sizeof(uint64_t), hipMemcpyHostToDevice, c->stream) !=
                    hipSuccess ||
                hipMemcpyAsync(dp, hp + j, (size_t)nb * sizeof(uint64_t), hipMemcpyHostToDevice, c->stream) !=
                    hipSuccess) {
                s = fail(PW_ERR_HIP, "x list copy failed");
                break;
            }
            s = eval_list_on(c, dx, 0, nb, eps, dr, c->stream, dp);
            if (s != PW_OK) break;
            if (hipMemcpyAsync(hres + j, dr, (size_t)nb * sizeof(FamilyRes), hipMemcpyDeviceToHost, c->stream) !=
                hipSuccess)
                s = fail(PW_ERR_HIP, "result copy failed");
        }
    }
    if (s == PW_OK && hipStreamSynchronize(c->stream) != hipSuccess) s = fail(PW_ERR_HIP, "synchronisation failed");
    s = restore(s);
    if (s != PW_OK) return s;
    for (int64_t j = 0; j < n_x; ++j) memcpy(out + seq[(size_t)j], hres + j, sizeof(FamilyRes));
    return PW_OK;
}

pw_status pw_set_precision(pw_ctx c, pw_prec prec) {
    pw_status s = check_ctx(c);
    if (s != PW_OK) return s;
    if (prec < PW_PREC_AUTO || prec > PW_PREC_BF16X2) return fail(PW_ERR_ARG, "unknown precision %d", (int)prec);
    if (prec == c->prec) return PW_OK;
    c->prec = prec;
    if (c->bound) {
        c->bound = false;   // re-plan (and re-carve) for the new arithmetic
        c->cdf_valid = false;
        s = prepare_workspace(c, c->n, c->dtype);
        if (s != PW_OK) return s;
        c->bound = true;
    }
    return PW_OK;
}

pw_status pw_set_progress(pw_ctx c, pw_progress_fn fn, void* user, double every_seconds) {
    pw_status s = check_ctx(c);
    if (s != PW_OK) return s;
    if (!(every_seconds >= 0.0)) return fail(PW_ERR_ARG, "every_seconds must be >= 0");
    c->progress = fn;
    c->progress_user = user;
    c->progress_every = every_seconds;
    return PW_OK;
}

pw_status pw_inject_fault(pw_ctx c, int cls) {
    pw_status s = check_ctx(c);
    if (s != PW_OK) return s;
    if (cls < FAULT_NONE || cls > FAULT_COPY) return fail(PW_ERR_ARG, "fault class %d outside [0, 3]", cls);
    c->fault_class = cls;
    return PW_OK;
}

pw_status pw_set_graphs(pw_ctx c, int enable) {
    pw_status s = check_ctx(c);
    if (s != PW_OK) return s;
    c->use_graphs = enable != 0;
    return PW_OK;
}

pw_status pw_set_moments(pw_ctx c, int max_alpha) {
    pw_status s = check_ctx(c);
    if (s != PW_OK) return s;
    if (max_alpha != 2 && max_alpha != 4) return fail(PW_ERR_ARG, "max_alpha must be 2 or 4, got %d", max_alpha);
    c->max_alpha = max_alpha;
    return PW_OK;
}

pw_status pw_timing_enable(pw_ctx c, int every) {
    pw_status s = check_ctx(c);
    if (s != PW_OK) return s;
    if (every < 0) return fail(PW_ERR_ARG, "every must be >= 0");
    c->timing_every = every;
    for (int k = 0; k < PW_KCLASSES; ++k) c->launches[k] = 0;
    return PW_OK;
}

pw_status pw_timing_read(pw_ctx c, int kclass, uint64_t* samples, double* total_ms, uint64_t* families) {
    pw_status s = check_ctx(c);
    if (s != PW_OK) return s;
    if (kclass < 0 || kclass >= PW_KCLASSES)
        return fail(PW_ERR_ARG, "kernel class %d outside [0, %d]", kclass, PW_KCLASSES - 1);
    for (auto& p : c->pending) {
        PW_HIP(hipEventSynchronize(p.b));
        float ms = 0.f;
        PW_HIP(hipEventElapsedTime(&ms, p.a, p.b));
        c->total_ms[p.kclass] += ms;
        c->samples[p.kclass] += 1;
        c->sampled_families[p.kclass] += (uint64_t)p.families;
        c->pool.push_back(p.a);
        c->pool.push_back(p.b);
    }
    c->pending.clear();
    if (samples) *samples = c->samples[kclass];
    if (total_ms) *total_ms = c->total_ms[kclass];
    if (families) *families = c->sampled_families[kclass];
    return PW_OK;
}

pw_status pw_timing_reset(pw_ctx c) {
    pw_status s = check_ctx(c);
    if (s != PW_OK) return s;
    uint64_t a;
    double b;
    s = pw_timing_read(c, 0, &a, &b, &a);
    if (s != PW_OK) return s;
    for (int k = 0; k < PW_KCLASSES; ++k) {
        c->total_ms[k] = 0;
        c->samples[k] = 0;
        c->sampled_families[k] = 0;
        c->launches[k] = 0;
    }
    return PW_OK;
}

}  // extern "C"
