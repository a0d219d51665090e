// pw_eval_x_noalloc: the families of a device list of x, for callers that cannot
// allocate device memory (code under HIP graph capture, tight serving loops).
//
// The kernels are those of pw_eval_x_device (product, transform passes, reductions,
// per-family finalisation, and for states of 16 MiB and more the sort by top bit and
// the tile-sharing groups of the first pass).  Their scratch (half spectra of the
// families in flight, final-pass partials, the sorted list and its results) lives in
// one file-scope device array of NOALLOC_SCRATCH_BYTES per GPU, held until the process
// ends.  Host code never uses the array's name as an address: on the first call on a
// device its address is taken once with hipGetSymbolAddress (that device current) and
// kept per device.  Every call on a GPU shares that GPU's array; overlapping calls on
// one GPU race.  Nothing in the array has to start at zero: every kernel writes what a
// later kernel of the same call reads.
#include "common.h"
#include "pauliwht.h"

#include <mutex>
#include <string>

namespace {

constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)128 << 20;
constexpr int MAX_DEVICES = 64;
constexpr int NOALLOC_MAX_LAUNCH = 256;   // families per launch (as the default workspace)
constexpr int FUSED_CHUNK = 4096;         // families per launch of single-workgroup plans

__device__ __align__(256) char scratch[NOALLOC_SCRATCH_BYTES];

std::mutex g_mu;
void* g_scratch[MAX_DEVICES] = {};

size_t al256(size_t v) { return (v + 255) & ~(size_t)255; }

pw_status nfail(pw_status s, const std::string& msg) {
    pw::last_error_ref() = msg;
    return s;
}

// Device address of this GPU's scratch array (resolved once per device, with it current).
pw_status scratch_of(int dev, char** out) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_scratch[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return nfail(PW_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch[dev] = p;
    }
    *out = (char*)g_scratch[dev];
    return PW_OK;
}

// Scratch layout of one call: launches of nb families, and (tile-sharing groups) the
// sorted copy of a list chunk, its order and its results.
struct NoallocLayout {
    size_t work, parts, xsort, perm, res2, total;
};

NoallocLayout noalloc_layout(const pw::Plan& P, size_t esz, int nb, bool grouped) {
    NoallocLayout L{};
    size_t off = 0;
    L.work = off;
    off += al256((size_t)nb * ((size_t)1 << P.nh) * esz);
    L.parts = off;
    off += al256((size_t)nb * (size_t)P.blocks_last * sizeof(pw::FamilyRes));
    if (grouped) {
        L.xsort = off;
        off += al256((size_t)pw::SORT_MAX * sizeof(uint64_t));
        L.perm = off;
        off += al256((size_t)pw::SORT_MAX * sizeof(uint32_t));
        L.res2 = off;
        off += al256((size_t)pw::SORT_MAX * sizeof(pw::FamilyRes));
    }
    L.total = off;
    return L;
}

}  // namespace

extern "C" pw_status pw_eval_x_noalloc(void* hip_stream, int n, pw_dtype dt, const void* dev_psi,
                                       const uint64_t* d_xs, int64_t nx, double eps, pw_xres* d_out) {
    if (dt != PW_C128 && dt != PW_C64) return nfail(PW_ERR_ARG, "unknown dtype " + std::to_string((int)dt));
    if (n < 1 || n > 32) return nfail(PW_ERR_RANGE, "n=" + std::to_string(n) + " outside [1, 32]");
    if (!dev_psi) return nfail(PW_ERR_ARG, "null state pointer");
    if ((uintptr_t)dev_psi & 255) return nfail(PW_ERR_ARG, "state must be 256-byte aligned");
    if (nx < 0) return nfail(PW_ERR_ARG, "negative count");
    if (nx > 0 && (!d_xs || !d_out)) return nfail(PW_ERR_ARG, "null array");
    if (!(eps >= 0.0 && eps < 1.0)) return nfail(PW_ERR_ARG, "eps outside [0, 1)");
    const bool dbl = dt == PW_C128;
    const size_t esz = dbl ? 16 : 8;
    const pw::Plan P = pw::make_plan(n, dbl);
    const bool grouped = !P.fused && pw::first_pass_group(P, dbl, 4) > 1;
    int nb = P.fused ? FUSED_CHUNK : NOALLOC_MAX_LAUNCH;
    if (!P.fused) {
        while (nb >= 1 && noalloc_layout(P, esz, nb, grouped).total > NOALLOC_SCRATCH_BYTES) nb /= 2;
        if (nb < 1)
            return nfail(PW_ERR_WORKSPACE,
                         "n=" + std::to_string(n) + (dbl ? " complex128" : " complex64") + " needs " +
                             std::to_string(noalloc_layout(P, esz, 1, grouped).total) +
                             " bytes of scratch for one family; the static scratch holds " +
                             std::to_string(NOALLOC_SCRATCH_BYTES) + " (complex64 n <= 24, complex128 n <= 23)");
    }
    if (nx == 0) return PW_OK;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return nfail(PW_ERR_HIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
    if (dev < 0 || dev >= MAX_DEVICES) return nfail(PW_ERR_RANGE, "device index above 63");
    char* base = nullptr;
    pw_status s = scratch_of(dev, &base);
    if (s != PW_OK) return s;
    hipStream_t st = (hipStream_t)hip_stream;
    pw::FamilyRes* out = reinterpret_cast<pw::FamilyRes*>(d_out);
#define NA_HIP(call)                                                                       \
    do {                                                                                   \
        hipError_t e_ = (call);                                                            \
        if (e_ != hipSuccess) return nfail(PW_ERR_HIP, std::string(#call ": ") + hipGetErrorString(e_)); \
    } while (0)
    if (P.fused) {
        for (int64_t i = 0; i < nx; i += nb) {
            const int m = (int)((nx - i) < nb ? (nx - i) : nb);
            NA_HIP(pw::eval_batch(P, dbl, 4, dev_psi, d_xs + i, 0, m, eps, nullptr, nullptr, out + i, st));
        }
        return PW_OK;
    }
    const NoallocLayout L = noalloc_layout(P, esz, nb, grouped);
    void* work = base + L.work;
    pw::FamilyRes* parts = reinterpret_cast<pw::FamilyRes*>(base + L.parts);
    if (!grouped) {
        for (int64_t i = 0; i < nx; i += nb) {
            const int m = (int)((nx - i) < nb ? (nx - i) : nb);
            NA_HIP(pw::eval_batch(P, dbl, 4, dev_psi, d_xs + i, 0, m, eps, work, parts, out + i, st));
        }
        return PW_OK;
    }
    // tile-sharing groups: each chunk of the list is evaluated in top-bit order and its
    // results are put back in list order (bitwise those of one family per launch)
    uint64_t* xs2 = reinterpret_cast<uint64_t*>(base + L.xsort);
    uint32_t* perm = reinterpret_cast<uint32_t*>(base + L.perm);
    pw::FamilyRes* r2 = reinterpret_cast<pw::FamilyRes*>(base + L.res2);
    for (int64_t i = 0; i < nx; i += pw::SORT_MAX) {
        const int m = (int)((nx - i) < pw::SORT_MAX ? (nx - i) : pw::SORT_MAX);
        NA_HIP(pw::sort_by_top_bit(d_xs + i, n, m, xs2, perm, st));
        for (int j = 0; j < m; j += nb) {
            const int k = (m - j) < nb ? (m - j) : nb;
            NA_HIP(pw::eval_batch(P, dbl, 4, dev_psi, xs2 + j, 0, k, eps, work, parts, r2 + j, st));
        }
        NA_HIP(pw::scatter_results(r2, perm, m, out + i, st));
    }
#undef NA_HIP
    return PW_OK;
}
