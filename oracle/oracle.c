/*
 * Plain FP64 CPU oracle for FWHT Pauli-string evaluation (Xiao & Ryu,
 * "Exponentially Accelerated Sampling of Pauli Strings for Nonstabilizerness").
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code with
 * the HIP library: it is a slow, obviously correct restatement of the paper's
 * definitions and of Algorithm 1, in double precision, with no blocking, no
 * fusion and no reordering beyond what those definitions state.
 *
 * Conventions (the paper leaves them open):
 *   - qubit j is bit j of the basis index (little endian);
 *   - the Hermitian Pauli of label (x, z) is P = i^{|x&z|} X^x Z^z, i.e. Y = iXZ
 *     on every qubit where both bits are set; then
 *     <psi|P|psi> = (-i)^{|x&z|} F_x(z) with F_x the Walsh-Hadamard transform of
 *     f_x(b) = conj(psi(b)) psi(b^x)  (Pauli labelling section, Eqs. for P_{x,z});
 *   - complex arrays are interleaved (re, im) doubles.
 *
 * Every exported function returns 0 on success and a negative value on bad
 * arguments.  Large loops use OpenMP.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

#define PWO_EXPORT __attribute__((visibility("default")))

typedef struct { double re, im; } cplx;

static inline cplx cmul(cplx a, cplx b) { cplx r = {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; return r; }
static inline cplx cconj(cplx a) { cplx r = {a.re, -a.im}; return r; }
static inline double cabs2(cplx a) { return a.re * a.re + a.im * a.im; }

/* Neumaier's compensated summation. */
typedef struct { double s, c; } nsum;
static inline void nadd(nsum* a, double v) {
    double t = a->s + v;
    if (fabs(a->s) >= fabs(v)) a->c += (a->s - t) + v; else a->c += (v - t) + a->s;
    a->s = t;
}
static inline double nval(const nsum* a) { return a->s + a->c; }


/* ------------------------------------------------------------------------ */
/* Brute force: the definition c_P = <psi|P|psi> for every Pauli string      */
/* (Pauli expansion paragraph; single-correlator cost O(2^N)).               */
/* ------------------------------------------------------------------------ */

/* Matrix element <b^x_j| sigma |b_j> of the single-qubit Pauli with bits (xj, zj):
 * (0,0)=I, (1,0)=X, (0,1)=Z, (1,1)=Y=[[0,-i],[i,0]]. */
static cplx pauli_elem(int xj, int zj, int bj) {
    cplx one = {1.0, 0.0};
    if (!xj && !zj) return one;                         /* I */
    if (xj && !zj) return one;                          /* X|b> = |1-b> */
    if (!xj && zj) { cplx r = {bj ? -1.0 : 1.0, 0.0}; return r; }   /* Z|b> = (-1)^b |b> */
    /* Y|0> = i|1>, Y|1> = -i|0> */
    { cplx r = {0.0, bj ? -1.0 : 1.0}; return r; }
}

/* c[x * 2^n + z] (real and imaginary part) for all 4^n strings; n <= 12.
 * P|b> = phase(b) |b^x>, phase(b) = prod_j <b_j^x_j|sigma_j|b_j>, built from two
 * half-register tables so that the O(8^n) loop is one multiply per term. */
PWO_EXPORT int pwo_bruteforce(int n, const double* psi_in, double* c_re, double* c_im) {
    if (n < 1 || n > 12 || !psi_in || !c_re || !c_im) return -1;
    const uint64_t d = 1ull << n;
    const cplx* psi = (const cplx*)psi_in;
    const int nl = n / 2, nh = n - nl;
    const uint64_t dl = 1ull << nl, dh = 1ull << nh;
    /* tab_lo[(xl, zl, bl)] = prod over low qubits; tab_hi likewise. */
    cplx* tlo = (cplx*)malloc(sizeof(cplx) * dl * dl * dl);
    cplx* thi = (cplx*)malloc(sizeof(cplx) * dh * dh * dh);
    if (!tlo || !thi) { free(tlo); free(thi); return -2; }
    for (uint64_t xl = 0; xl < dl; ++xl)
        for (uint64_t zl = 0; zl < dl; ++zl)
            for (uint64_t bl = 0; bl < dl; ++bl) {
                cplx ph = {1.0, 0.0};
                for (int j = 0; j < nl; ++j)
                    ph = cmul(ph, pauli_elem((xl >> j) & 1, (zl >> j) & 1, (bl >> j) & 1));
                tlo[(xl * dl + zl) * dl + bl] = ph;
            }
    for (uint64_t xh = 0; xh < dh; ++xh)
        for (uint64_t zh = 0; zh < dh; ++zh)
            for (uint64_t bh = 0; bh < dh; ++bh) {
                cplx ph = {1.0, 0.0};
                for (int j = 0; j < nh; ++j)
                    ph = cmul(ph, pauli_elem((xh >> j) & 1, (zh >> j) & 1, (bh >> j) & 1));
                thi[(xh * dh + zh) * dh + bh] = ph;
            }
    #pragma omp parallel for schedule(dynamic, 1)
    for (int64_t xz = 0; xz < (int64_t)(d * d); ++xz) {
        uint64_t x = (uint64_t)xz >> n, z = (uint64_t)xz & (d - 1);
        uint64_t xl = x & (dl - 1), xh = x >> nl, zl = z & (dl - 1), zh = z >> nl;
        const cplx* tl = tlo + (xl * dl + zl) * dl;
        const cplx* th = thi + (xh * dh + zh) * dh;
        /* <psi|P|psi> = sum_b conj(psi(b^x)) phase(b) psi(b) */
        double sr = 0.0, si = 0.0;
        for (uint64_t b = 0; b < d; ++b) {
            cplx ph = cmul(tl[b & (dl - 1)], th[b >> nl]);
            cplx t = cmul(cconj(psi[b ^ x]), cmul(ph, psi[b]));
            sr += t.re; si += t.im;
        }
        c_re[xz] = sr; c_im[xz] = si;
    }
    free(tlo); free(thi);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Algorithm 1 (End Matter, FWHT-based Pauli sampling), per family x.        */
/* ------------------------------------------------------------------------ */

/* In-place unnormalised Walsh-Hadamard transform, textbook stage order
 * h = 1, 2, 4, ...: (a, b) -> (a + b, a - b) (the (sqrt2 H)^{\otimes N} of the
 * FWHT paragraph).  `par` enables OpenMP inside each stage. */
static void fwht_inplace(cplx* v, uint64_t d, int par) {
    for (uint64_t h = 1; h < d; h <<= 1) {
        #pragma omp parallel for if (par) schedule(static)
        for (int64_t i0 = 0; i0 < (int64_t)(d >> 1); ++i0) {
            uint64_t lo = (uint64_t)i0 & (h - 1), hi = ((uint64_t)i0 >> __builtin_ctzll(h)) ;
            uint64_t i = hi * (h << 1) + lo, j = i + h;
            cplx a = v[i], b = v[j];
            v[i].re = a.re + b.re; v[i].im = a.im + b.im;
            v[j].re = a.re - b.re; v[j].im = a.im - b.im;
        }
    }
}

/* f_x(b) = conj(psi(b)) psi(b ^ x) for all b (Algorithm 1, product step). */
static void form_fx(const cplx* psi, uint64_t d, uint64_t x, cplx* f, int par) {
    #pragma omp parallel for if (par) schedule(static)
    for (int64_t b = 0; b < (int64_t)d; ++b) f[b] = cmul(cconj(psi[b]), psi[(uint64_t)b ^ x]);
}

typedef struct {
    double p;        /* m_{1;x} = sum_z |F|^2 / d                      */
    double ent;      /* sum_z |F|^2 log2 |F|^2  (0 log 0 = 0)           */
    double m[7];     /* m_{alpha;x} for alpha = 2..8                    */
    uint64_t nu;     /* #{z : ||F| - 1| < eps}                           */
    double gap;      /* max{|F| : |F| < 1 - eps}, -1 if none            */
    /* sums over z that size first-order rounding bounds of a reduced-precision
     * evaluation of the same family (not part of Algorithm 1):
     * sum |F|, |F|^3, |F|^5, |F|^7, |2|F| log2|F|^2 + 2|F|/ln 2|, ||F|^2 log2 |F|^2| */
    double bsum[6];
} xres;

/* Reductions of Algorithm 1 over one spectrum F_x (nullity count, partial
 * moments) plus the Shannon term needed for alpha = 1. */
static void reduce_spectrum(const cplx* F, int n, double eps, int max_alpha, xres* r, int par) {
    const uint64_t d = 1ull << n;
    nsum sp = {0, 0}, se = {0, 0};
    nsum sm[7];
    memset(sm, 0, sizeof sm);
    uint64_t nu = 0;
    double gap = -1.0;
    nsum sb[6];
    memset(sb, 0, sizeof sb);
    #pragma omp parallel if (par)
    {
        nsum lp = {0, 0}, le = {0, 0}, lm[7], lb[6];
        memset(lm, 0, sizeof lm);
        memset(lb, 0, sizeof lb);
        uint64_t lnu = 0;
        double lgap = -1.0;
        #pragma omp for schedule(static) nowait
        for (int64_t z = 0; z < (int64_t)d; ++z) {
            double a2 = cabs2(F[z]);
            double a = sqrt(a2);
            if (fabs(a - 1.0) < eps) ++lnu;
            else if (a < 1.0 - eps && a > lgap) lgap = a;
            nadd(&lp, a2);
            if (a2 > 0.0) nadd(&le, a2 * log2(a2));
            double pw = a2;
            for (int al = 2; al <= max_alpha; ++al) { pw *= a2; nadd(&lm[al - 2], pw); }
            nadd(&lb[0], a);
            nadd(&lb[1], a * a2);
            nadd(&lb[2], a * a2 * a2);
            nadd(&lb[3], a * a2 * a2 * a2);
            if (a2 > 0.0) {
                nadd(&lb[4], fabs(2.0 * a * log2(a2) + 2.0 * a / log(2.0)));
                nadd(&lb[5], fabs(a2 * log2(a2)));
            }
        }
        #pragma omp critical
        {
            nadd(&sp, nval(&lp)); nadd(&se, nval(&le));
            for (int al = 2; al <= max_alpha; ++al) nadd(&sm[al - 2], nval(&lm[al - 2]));
            for (int k = 0; k < 6; ++k) nadd(&sb[k], nval(&lb[k]));
            nu += lnu;
            if (lgap > gap) gap = lgap;
        }
    }
    for (int k = 0; k < 6; ++k) r->bsum[k] = nval(&sb[k]);
    r->p = ldexp(nval(&sp), -n);
    r->ent = nval(&se);
    for (int al = 2; al <= 8; ++al) r->m[al - 2] = (al <= max_alpha) ? ldexp(nval(&sm[al - 2]), -n * al) : 0.0;
    r->nu = nu;
    r->gap = gap;
}

/* Per-family results for a list of x (the per-family steps of Algorithm 1: product,
 * transform, nullity count and moments, plus the Shannon term).  Outputs are arrays of length nx; m has nx*(max_alpha-1)
 * entries, alpha-major within each x. */
static int eval_x_impl(int n, const double* psi_in, const uint64_t* xs, int64_t nx, double eps,
                       int max_alpha, double* p, double* ent, double* m, uint64_t* nu, double* gap, double* bsum) {
    if (n < 1 || n > 34 || !psi_in || !xs || nx < 0 || max_alpha < 2 || max_alpha > 8) return -1;
    const uint64_t d = 1ull << n;
    for (int64_t i = 0; i < nx; ++i) if (xs[i] >= d) return -1;
    const cplx* psi = (const cplx*)psi_in;
    const int outer = (n <= 16);
    if (outer) {
        #pragma omp parallel
        {
            cplx* f = (cplx*)malloc(sizeof(cplx) * d);
            #pragma omp for schedule(dynamic, 1)
            for (int64_t i = 0; i < nx; ++i) {
                xres r;
                form_fx(psi, d, xs[i], f, 0);
                fwht_inplace(f, d, 0);
                reduce_spectrum(f, n, eps, max_alpha, &r, 0);
                if (p) p[i] = r.p;
                if (ent) ent[i] = r.ent;
                if (m) for (int al = 2; al <= max_alpha; ++al) m[i * (max_alpha - 1) + (al - 2)] = r.m[al - 2];
                if (nu) nu[i] = r.nu;
                if (gap) gap[i] = r.gap;
                if (bsum) memcpy(bsum + 6 * i, r.bsum, sizeof r.bsum);
            }
            free(f);
        }
    } else {
        cplx* f = (cplx*)malloc(sizeof(cplx) * d);
        if (!f) return -2;
        for (int64_t i = 0; i < nx; ++i) {
            xres r;
            form_fx(psi, d, xs[i], f, 1);
            fwht_inplace(f, d, 1);
            reduce_spectrum(f, n, eps, max_alpha, &r, 1);
            if (p) p[i] = r.p;
            if (ent) ent[i] = r.ent;
            if (m) for (int al = 2; al <= max_alpha; ++al) m[i * (max_alpha - 1) + (al - 2)] = r.m[al - 2];
            if (nu) nu[i] = r.nu;
            if (gap) gap[i] = r.gap;
            if (bsum) memcpy(bsum + 6 * i, r.bsum, sizeof r.bsum);
        }
        free(f);
    }
    return 0;
}

PWO_EXPORT int pwo_eval_x(int n, const double* psi_in, const uint64_t* xs, int64_t nx, double eps,
                          int max_alpha, double* p, double* ent, double* m, uint64_t* nu, double* gap) {
    return eval_x_impl(n, psi_in, xs, nx, eps, max_alpha, p, ent, m, nu, gap, NULL);
}

/* pwo_eval_x plus, per x, the six sums of xres.bsum (6 doubles per x in bsum), from the
 * same transform: what first-order rounding bounds of a reduced-precision evaluation of
 * the family need. */
PWO_EXPORT int pwo_eval_x_sums(int n, const double* psi_in, const uint64_t* xs, int64_t nx, double eps,
                               int max_alpha, double* p, double* ent, double* m, uint64_t* nu, double* gap,
                               double* bsum) {
    if (!bsum) return -1;
    return eval_x_impl(n, psi_in, xs, nx, eps, max_alpha, p, ent, m, nu, gap, bsum);
}

/* The raw transform F_x(z) for one x (complex, length 2^n). */
PWO_EXPORT int pwo_spectrum(int n, const double* psi_in, uint64_t x, double* F_out) {
    if (n < 1 || n > 30 || !psi_in || !F_out || x >= (1ull << n)) return -1;
    const uint64_t d = 1ull << n;
    form_fx((const cplx*)psi_in, d, x, (cplx*)F_out, n > 16);
    fwht_inplace((cplx*)F_out, d, n > 16);
    return 0;
}

/* Algorithm 1 in full: sweep every x, accumulate m_alpha and nu_cnt
 * (compensated), and the Shannon sum for M_1.  Outputs:
 *   S[alpha-2] = sum_x m_{alpha;x}, alpha = 2..max_alpha;
 *   *L = sum_x ent_x;  *P = sum_x p(x) (equals 1 for a normalised state);
 *   *nu_cnt = sum_x nu_x.  Per-x arrays may be NULL. */
PWO_EXPORT int pwo_alg1(int n, const double* psi_in, double eps, int max_alpha,
                        double* S, double* L, double* P, uint64_t* nu_cnt,
                        double* p_x, double* ent_x, double* m_x, uint64_t* nu_x, double* gap_x) {
    if (n < 1 || n > 24 || !psi_in || max_alpha < 2 || max_alpha > 8 || !S || !L || !P || !nu_cnt) return -1;
    const uint64_t d = 1ull << n;
    const int na = max_alpha - 1;
    uint64_t* xs = (uint64_t*)malloc(sizeof(uint64_t) * d);
    double* pp = p_x ? p_x : (double*)malloc(sizeof(double) * d);
    double* ee = ent_x ? ent_x : (double*)malloc(sizeof(double) * d);
    double* mm = m_x ? m_x : (double*)malloc(sizeof(double) * d * na);
    uint64_t* vv = nu_x ? nu_x : (uint64_t*)malloc(sizeof(uint64_t) * d);
    double* gg = gap_x ? gap_x : (double*)malloc(sizeof(double) * d);
    if (!xs || !pp || !ee || !mm || !vv || !gg) return -2;
    for (uint64_t x = 0; x < d; ++x) xs[x] = x;
    int rc = pwo_eval_x(n, psi_in, xs, (int64_t)d, eps, max_alpha, pp, ee, mm, vv, gg);
    if (rc == 0) {
        nsum sa[7], sl = {0, 0}, sp = {0, 0};
        memset(sa, 0, sizeof sa);
        uint64_t cnt = 0;
        for (uint64_t x = 0; x < d; ++x) {            /* fixed x order */
            for (int a = 0; a < na; ++a) nadd(&sa[a], mm[x * na + a]);
            nadd(&sl, ee[x]); nadd(&sp, pp[x]);
            cnt += vv[x];
        }
        for (int a = 0; a < na; ++a) S[a] = nval(&sa[a]);
        *L = nval(&sl); *P = nval(&sp); *nu_cnt = cnt;
    }
    free(xs);
    if (!p_x) free(pp);
    if (!ent_x) free(ee);
    if (!m_x) free(mm);
    if (!nu_x) free(vv);
    if (!gap_x) free(gg);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Exact x-marginal p(x) = sum_z c^2/d over the family = sum_b q(b) q(b^x),  */
/* q = |psi|^2 (Parseval applied to the family's transform).                 */
/* ------------------------------------------------------------------------ */
PWO_EXPORT int pwo_marginal(int n, const double* psi_in, const uint64_t* xs, int64_t nx, double* p) {
    if (n < 1 || n > 34 || !psi_in || !xs || !p || nx < 0) return -1;
    const uint64_t d = 1ull << n;
    const cplx* psi = (const cplx*)psi_in;
    for (int64_t i = 0; i < nx; ++i) {
        uint64_t x = xs[i];
        if (x >= d) return -1;
        double s = 0.0;
        #pragma omp parallel for reduction(+ : s) schedule(static) if (n > 14)
        for (int64_t b = 0; b < (int64_t)d; ++b) s += cabs2(psi[b]) * cabs2(psi[(uint64_t)b ^ x]);
        p[i] = s;
    }
    return 0;
}

/* Squared norm in FP64. */
PWO_EXPORT double pwo_norm2(int n, const double* psi_in) {
    const uint64_t d = 1ull << n;
    const cplx* psi = (const cplx*)psi_in;
    double s = 0.0;
    #pragma omp parallel for reduction(+ : s) schedule(static) if (n > 14)
    for (int64_t b = 0; b < (int64_t)d; ++b) s += cabs2(psi[b]);
    return s;
}

/* ------------------------------------------------------------------------ */
/* Gate application (Clifford preconditioning and state preparation).        */
/* kinds[g] = 2: dense 4x4 on (q0, q1), local index b_{q0} + 2 b_{q1};       */
/* kinds[g] = 1: diagonal (d0, d1) on q0, stored in mats[g][0][0..1].        */
/* mats: 16 complex per gate, row-major.                                     */
/* ------------------------------------------------------------------------ */
PWO_EXPORT int pwo_apply_gates(int n, double* psi_io, int ng, const int* kinds, const int* qubits,
                               const double* mats_in) {
    if (n < 1 || n > 34 || !psi_io || ng < 0 || (ng > 0 && (!kinds || !qubits || !mats_in))) return -1;
    const uint64_t d = 1ull << n;
    cplx* psi = (cplx*)psi_io;
    const cplx* mats = (const cplx*)mats_in;
    for (int g = 0; g < ng; ++g) {
        const cplx* u = mats + 16 * g;
        int q0 = qubits[2 * g], q1 = qubits[2 * g + 1];
        if (q0 < 0 || q0 >= n) return -1;
        if (kinds[g] == 2) {
            if (q1 < 0 || q1 >= n || q1 == q0) return -1;
            uint64_t m0 = 1ull << q0, m1 = 1ull << q1;
            #pragma omp parallel for schedule(static) if (n > 14)
            for (int64_t b = 0; b < (int64_t)d; ++b) {
                if ((uint64_t)b & (m0 | m1)) continue;
                uint64_t idx[4] = {(uint64_t)b, (uint64_t)b | m0, (uint64_t)b | m1, (uint64_t)b | m0 | m1};
                cplx in[4], out[4];
                for (int j = 0; j < 4; ++j) in[j] = psi[idx[j]];
                for (int r = 0; r < 4; ++r) {
                    cplx s = {0.0, 0.0};
                    for (int c = 0; c < 4; ++c) { cplx t = cmul(u[4 * r + c], in[c]); s.re += t.re; s.im += t.im; }
                    out[r] = s;
                }
                for (int j = 0; j < 4; ++j) psi[idx[j]] = out[j];
            }
        } else if (kinds[g] == 1) {
            uint64_t m0 = 1ull << q0;
            cplx d0 = u[0], d1 = u[1];
            #pragma omp parallel for schedule(static) if (n > 14)
            for (int64_t b = 0; b < (int64_t)d; ++b) psi[b] = cmul(((uint64_t)b & m0) ? d1 : d0, psi[b]);
        } else {
            return -1;
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) and the two x samplers. */
/* ------------------------------------------------------------------------ */
static void philox_round(uint32_t c[4], const uint32_t k[2]) {
    uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
    uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t n0 = hi1 ^ c[1] ^ k[0], n2 = hi0 ^ c[3] ^ k[1];
    c[0] = n0; c[1] = lo1; c[2] = n2; c[3] = lo0;
}

PWO_EXPORT void pwo_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
    uint32_t c[4] = {ctr[0], ctr[1], ctr[2], ctr[3]};
    uint32_t k[2] = {key[0], key[1]};
    for (int r = 0; r < 10; ++r) {
        philox_round(c, k);
        k[0] += 0x9E3779B9u; k[1] += 0xBB67AE85u;
    }
    /* round r uses key + r*(W0, W1); the bump after the last round is unused */
    out[0] = c[0]; out[1] = c[1]; out[2] = c[2]; out[3] = c[3];
}

#define PWO_STREAM_UNIFORM 0x554E4946u   /* "UNIF" */
#define PWO_STREAM_MARGINAL 0x4D415247u  /* "MARG" */
#define PWO_MAX_ATTEMPTS 64

static void philox_words(uint64_t seed, uint64_t g, uint32_t attempt, uint32_t stream, uint64_t* W0, uint64_t* W1) {
    uint32_t ctr[4] = {(uint32_t)g, (uint32_t)(g >> 32), attempt, stream};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t w[4];
    pwo_philox4x32_10(ctr, key, w);
    *W0 = ((uint64_t)w[1] << 32) | w[0];
    *W1 = ((uint64_t)w[3] << 32) | w[2];
}

/* The paper's Monte Carlo draw: x uniform on F_2^N minus {0}
 * (Monte Carlo section: "sample the remaining values uniformly").
 * Sample i of the list is x = 1 + floor(W0 * (2^n - 1) / 2^64) with W0 the first
 * 64-bit word of Philox(ctr = (offset+i, 0, UNIF), key = seed). */
PWO_EXPORT int pwo_sample_uniform_nz(int n, uint64_t seed, uint64_t offset, int64_t count, uint64_t* xs) {
    if (n < 1 || n > 34 || count < 0 || !xs) return -1;
    const uint64_t m = (1ull << n) - 1;
    for (int64_t i = 0; i < count; ++i) {
        uint64_t W0, W1;
        philox_words(seed, offset + (uint64_t)i, 0, PWO_STREAM_UNIFORM, &W0, &W1);
        xs[i] = 1 + (uint64_t)(((unsigned __int128)W0 * m) >> 64);
    }
    return 0;
}

/* Inverse-CDF draw restricted to [lo, hi]: smallest k there with C[k] > t, or hi. */
static uint64_t cdf_search_in(const double* C, uint64_t lo, uint64_t hi, double t) {
    while (lo < hi) {
        uint64_t mid = lo + ((hi - lo) >> 1);
        if (C[mid] > t) hi = mid; else lo = mid + 1;
    }
    return lo;
}

/* Inverse-CDF draw: smallest k with C[k] > t. */
static uint64_t cdf_search(const double* C, uint64_t d, double t) { return cdf_search_in(C, 0, d - 1, t); }

/* A pair b1 != b2 drawn directly from the law of two independent draws from q
 * conditioned on being different: b1 from w(b) = q(b) (T - q(b)) (the chance that b
 * comes first and the second draw is not b; Cw its inclusive prefix sum), then b2
 * from q with b1 removed, i.e. the point u2 (T - q(b1)) of the remaining mass mapped
 * past b1's own interval of C.  Returns b1 ^ b2 (never 0), or 0 when w vanishes
 * (q a point mass). */
static uint64_t draw_distinct_pair(const double* C, const double* Cw, uint64_t d, double u1, double u2) {
    const double T = C[d - 1], Tw = Cw[d - 1];
    if (!(Tw > 0.0)) return 0;
    const uint64_t b1 = cdf_search(Cw, d, u1 * Tw);
    const double B = b1 ? C[b1 - 1] : 0.0;      /* mass below b1 */
    const double t = u2 * (T - (C[b1] - B));    /* a point of the mass without b1 */
    uint64_t b2;
    if (b1 > 0 && (t < B || b1 == d - 1)) b2 = cdf_search_in(C, 0, b1 - 1, t);
    else b2 = cdf_search_in(C, b1 + 1, d - 1, C[b1] + (t - B));
    return b1 ^ b2;
}

/* Inclusive prefix sums of q = |psi|^2 (C) and of w = q (T - q), T = C[d-1] (Cw). */
static void build_cdfs(const cplx* psi, uint64_t d, double* C, double* Cw) {
    double run = 0.0;
    for (uint64_t b = 0; b < d; ++b) { run += cabs2(psi[b]); C[b] = run; }
    const double T = C[d - 1];
    run = 0.0;
    for (uint64_t b = 0; b < d; ++b) { const double q = cabs2(psi[b]); run += q * (T - q); Cw[b] = run; }
}

/* Draws from the exact x-marginal p(x) = sum_b q(b) q(b^x), conditioned on x != 0:
 * x = b1 ^ b2 with b1, b2 independent draws from q = |psi|^2 (since the XOR of two
 * independent draws from q has exactly this law), redrawn while x == 0.
 * Attempt a of sample i uses Philox(ctr = (offset+i, a, MARG), key = seed):
 * u1 = (W0 >> 11) 2^-53, u2 = (W1 >> 11) 2^-53, b_j = smallest k with
 * C[k] > u_j C[d-1], C the inclusive prefix sum of q.  A sample that is still 0
 * after 64 attempts takes the words of attempt 64 and draw_distinct_pair, which has
 * the same conditional law, so the output law is exact whatever p(0) < 1.  The
 * return value counts samples left at 0 (only when q is a point mass).  Also
 * returns, if C_out is given, the prefix sums used (C_out[0..d): C; C_out[d..2d): Cw). */
PWO_EXPORT int64_t pwo_sample_marginal_nz(int n, const double* psi_in, uint64_t seed, uint64_t offset,
                                          int64_t count, uint64_t* xs, double* C_out) {
    if (n < 1 || n > 30 || count < 0 || !xs || !psi_in) return -1;
    const uint64_t d = 1ull << n;
    const cplx* psi = (const cplx*)psi_in;
    double* C = C_out ? C_out : (double*)malloc(sizeof(double) * 2 * d);
    if (!C) return -2;
    double* Cw = C + d;
    build_cdfs(psi, d, C, Cw);
    const double T = C[d - 1];
    int64_t failed = 0;
    for (int64_t i = 0; i < count; ++i) {
        uint64_t x = 0;
        for (uint32_t a = 0; a < PWO_MAX_ATTEMPTS && x == 0; ++a) {
            uint64_t W0, W1;
            philox_words(seed, offset + (uint64_t)i, a, PWO_STREAM_MARGINAL, &W0, &W1);
            double u1 = (double)(W0 >> 11) * 0x1.0p-53, u2 = (double)(W1 >> 11) * 0x1.0p-53;
            uint64_t b1 = cdf_search(C, d, u1 * T), b2 = cdf_search(C, d, u2 * T);
            x = b1 ^ b2;
        }
        if (x == 0) {
            uint64_t W0, W1;
            philox_words(seed, offset + (uint64_t)i, PWO_MAX_ATTEMPTS, PWO_STREAM_MARGINAL, &W0, &W1);
            x = draw_distinct_pair(C, Cw, d, (double)(W0 >> 11) * 0x1.0p-53, (double)(W1 >> 11) * 0x1.0p-53);
        }
        if (x == 0) ++failed;
        xs[i] = x;
    }
    if (!C_out) free(C);
    return failed;
}

/* The direct distinct-pair law alone (the words of attempt 64 for every sample), so
 * that tests can pin it on states where the redraw loop would rarely reach it.
 * Returns the number of samples left at 0. */
PWO_EXPORT int64_t pwo_sample_distinct_pairs(int n, const double* psi_in, uint64_t seed, int64_t count, uint64_t* xs) {
    if (n < 1 || n > 30 || count < 0 || !xs || !psi_in) return -1;
    const uint64_t d = 1ull << n;
    double* C = (double*)malloc(sizeof(double) * 2 * d);
    if (!C) return -2;
    build_cdfs((const cplx*)psi_in, d, C, C + d);
    int64_t failed = 0;
    for (int64_t i = 0; i < count; ++i) {
        uint64_t W0, W1;
        philox_words(seed, (uint64_t)i, PWO_MAX_ATTEMPTS, PWO_STREAM_MARGINAL, &W0, &W1);
        xs[i] = draw_distinct_pair(C, C + d, d, (double)(W0 >> 11) * 0x1.0p-53, (double)(W1 >> 11) * 0x1.0p-53);
        if (xs[i] == 0) ++failed;
    }
    free(C);
    return failed;
}

/* ------------------------------------------------------------------------ */
/* Mixed-state SRE of the reduced state on the first n_a qubits (Supplemental */
/* Material, mixed states, Eq. Msre-mixed): for every x_A,                    */
/*   h(a) = sum_e conj(psi(a, e)) psi(a ^ x_A, e),  b = a + 2^{n_a} e,        */
/* then an n_a-bit FWHT over a gives every c_P with P supported on A.         */
/* Outputs W[alpha-2] = sum_P |c_P|^{2 alpha} / d_A^alpha (alpha = 2..4),     */
/* *purity = sum_P |c_P|^2 / d_A = Tr rho_A^2, *L = sum_P c^2 log2 c^2.       */
/* ------------------------------------------------------------------------ */
PWO_EXPORT int pwo_mixed(int n, const double* psi_in, int n_a, double* W, double* purity, double* L) {
    if (n < 1 || n > 30 || n_a < 1 || n_a > n || n_a > 16 || !psi_in || !W || !purity || !L) return -1;
    const cplx* psi = (const cplx*)psi_in;
    const uint64_t dA = 1ull << n_a, dE = 1ull << (n - n_a);
    nsum sw[3], sp = {0, 0}, sl = {0, 0};
    memset(sw, 0, sizeof sw);
    cplx* h = (cplx*)malloc(sizeof(cplx) * dA);
    if (!h) return -2;
    for (uint64_t xa = 0; xa < dA; ++xa) {
        #pragma omp parallel for schedule(static)
        for (int64_t a = 0; a < (int64_t)dA; ++a) {
            double sr = 0.0, si = 0.0;
            for (uint64_t e = 0; e < dE; ++e) {
                cplx t = cmul(cconj(psi[(uint64_t)a + (e << n_a)]), psi[((uint64_t)a ^ xa) + (e << n_a)]);
                sr += t.re; si += t.im;
            }
            h[a].re = sr; h[a].im = si;
        }
        fwht_inplace(h, dA, 0);
        for (uint64_t z = 0; z < dA; ++z) {
            double a2 = cabs2(h[z]);
            nadd(&sp, a2);
            if (a2 > 0.0) nadd(&sl, a2 * log2(a2));
            double pw = a2;
            for (int al = 2; al <= 4; ++al) { pw *= a2; nadd(&sw[al - 2], pw); }
        }
    }
    free(h);
    for (int al = 2; al <= 4; ++al) W[al - 2] = ldexp(nval(&sw[al - 2]), -n_a * al);
    *purity = ldexp(nval(&sp), -n_a);
    *L = nval(&sl);
    return 0;
}
