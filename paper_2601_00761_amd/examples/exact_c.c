/*
 * Exact enumeration through the C ABI alone (no Python, no torch): reads a state
 * vector from a file, uploads it into a device buffer allocated with the HIP runtime,
 * runs pw_exact and reports the results.
 *
 * As a program:  exact_c <n_qubits> <dtype: 0 = complex128, 1 = complex64> <file> <eps>
 * prints one "key value" pair a line.  The file holds the 2^n amplitudes as
 * interleaved (re, im) in the given dtype.  Exit status: 0 on success, 1 on a usage or
 * I/O error, 2 on a library error.  Built without main (-DEXACT_C_NO_MAIN) the same code
 * is the function exact_c_run, for callers that load it as a shared object.
 */
#define __HIP_PLATFORM_AMD__ 1
#include <hip/hip_runtime_api.h>
#include <stdio.h>
#include <stdlib.h>

#include "pauliwht.h"

/* out[0..9] = status, <psi|psi>, S_2, S_3, S_4, M_1, M_2, nu_cnt, nullity, families.
 * Returns 0, 1 (usage or I/O) or 2 (library error; the message is pw_last_error()). */
__attribute__((visibility("default"))) int exact_c_run(int n, int dtype, const char* path, double eps,
                                                       double* out) {
    if (n < 1 || n > 26 || !path || !out) return 1;
    const pw_dtype dt = dtype ? PW_C64 : PW_C128;
    const size_t bytes = ((size_t)1 << n) * (dt == PW_C64 ? 8 : 16);
    void* host = malloc(bytes);
    FILE* f = fopen(path, "rb");
    const int ok = host && f && fread(host, 1, bytes, f) == bytes;
    if (f) fclose(f);
    void* dev = NULL;
    if (!ok || hipMalloc(&dev, bytes) != hipSuccess) {
        free(host);
        return 1;
    }
    pw_ctx ctx = NULL;
    double nrm = 0.0;
    pw_result r;
    pw_status s = pw_ctx_create(&ctx, 0, NULL);
    if (s == PW_OK) s = pw_state_upload(ctx, n, dt, host, dev, &nrm);
    if (s == PW_OK || s == PW_ERR_TOLERANCE) s = pw_exact(ctx, eps, &r);
    const int rc = (s == PW_OK || s == PW_ERR_TOLERANCE) ? 0 : 2;
    if (rc == 0) {
        out[0] = (double)s;
        out[1] = nrm;
        out[2] = r.S[0];
        out[3] = r.S[1];
        out[4] = r.S[2];
        out[5] = r.M1;
        out[6] = r.M[0];
        out[7] = (double)r.nu_cnt;
        out[8] = r.nullity;
        out[9] = (double)r.n_samples;
    }
    if (ctx) pw_ctx_destroy(ctx);
    (void)hipFree(dev);
    free(host);
    return rc;
}

#ifndef EXACT_C_NO_MAIN
int main(int argc, char** argv) {
    if (argc != 5) {
        fprintf(stderr, "usage: %s n dtype file eps\n", argv[0]);
        return 1;
    }
    double v[10];
    const int rc = exact_c_run(atoi(argv[1]), atoi(argv[2]), argv[3], atof(argv[4]), v);
    if (rc == 2) fprintf(stderr, "pauliwht error: %s\n", pw_last_error());
    if (rc) return rc;
    const char* key[10] = {"status", "norm2", "S2", "S3", "S4", "M1", "M2", "nu_cnt", "nullity", "families"};
    for (int i = 0; i < 10; ++i) printf("%s %.17g\n", key[i], v[i]);
    return 0;
}
#endif
