/* Plain-C use of libmr1l (no Python, no PyTorch): read a transform problem from raw little-endian
 * files, run one forward and one adjoint multiple rank-1 lattice FFT (Alg. 2, complex128) on
 * device 0, and write the results.
 *
 *   c_abi_example DIR
 *   DIR/shape    int64 [4]: d, n, L, sum_l M_l
 *   DIR/freqs    int32 [n][d]        DIR/M  int64 [L]        DIR/z  int64 [L][d]
 *   DIR/samples  double [sum M][2]   DIR/coeffs  double [n][2]
 * writes DIR/coeffs_out (forward of samples) and DIR/samples_out (adjoint of coeffs). */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include <hip/hip_runtime_api.h>

#include "mr1l.h"

static void* slurp(const char* dir, const char* name, size_t want) {
    char path[4096];
    snprintf(path, sizeof path, "%s/%s", dir, name);
    FILE* fh = fopen(path, "rb");
    if (!fh) return NULL;
    void* buf = malloc(want ? want : 1);
    size_t got = buf ? fread(buf, 1, want, fh) : 0;
    fclose(fh);
    if (got != want) {
        free(buf);
        return NULL;
    }
    return buf;
}

static int dump(const char* dir, const char* name, const void* buf, size_t bytes) {
    char path[4096];
    snprintf(path, sizeof path, "%s/%s", dir, name);
    FILE* fh = fopen(path, "wb");
    if (!fh) return 1;
    size_t put = fwrite(buf, 1, bytes, fh);
    fclose(fh);
    return put != bytes;
}

#define CHECK(call)                                                                        \
    do {                                                                                   \
        mr1l_status st_ = (call);                                                          \
        if (st_ != MR1L_OK && st_ != MR1L_WARN_UNCOVERED) {                                \
            fprintf(stderr, "%s failed (%d): %s\n", #call, (int)st_, mr1l_last_error());   \
            return 1;                                                                      \
        }                                                                                  \
    } while (0)

int main(int argc, char** argv) {
    if (argc != 2) {
        fprintf(stderr, "usage: %s DIR\n", argv[0]);
        return 2;
    }
    const char* dir = argv[1];
    int64_t* shape = (int64_t*)slurp(dir, "shape", 4 * sizeof(int64_t));
    if (!shape) return 2;
    const int d = (int)shape[0], L = (int)shape[2];
    const int64_t n = shape[1], sm = shape[3];
    int32_t* freqs = (int32_t*)slurp(dir, "freqs", (size_t)n * d * sizeof(int32_t));
    int64_t* M = (int64_t*)slurp(dir, "M", (size_t)L * sizeof(int64_t));
    int64_t* z = (int64_t*)slurp(dir, "z", (size_t)L * d * sizeof(int64_t));
    double* samples = (double*)slurp(dir, "samples", (size_t)sm * 16);
    double* coeffs = (double*)slurp(dir, "coeffs", (size_t)n * 16);
    if (!freqs || !M || !z || !samples || !coeffs) return 2;

    void *dy = NULL, *dc = NULL, *dc_in = NULL, *dy_out = NULL;
    if (hipMalloc(&dy, (size_t)sm * 16) != hipSuccess || hipMalloc(&dc, (size_t)n * 16) != hipSuccess ||
        hipMalloc(&dc_in, (size_t)n * 16) != hipSuccess || hipMalloc(&dy_out, (size_t)sm * 16) != hipSuccess)
        return 3;
    if (hipMemcpy(dy, samples, (size_t)sm * 16, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(dc_in, coeffs, (size_t)n * 16, hipMemcpyHostToDevice) != hipSuccess)
        return 3;

    mr1l_plan_t plan = NULL;
    CHECK(mr1l_plan(d, n, freqs, L, M, z, MR1L_C128, MR1L_W_PAPER, 1, 0, &plan));
    CHECK(mr1l_forward(plan, dy, dc, NULL));
    CHECK(mr1l_adjoint(plan, dc_in, dy_out, NULL));
    if (hipDeviceSynchronize() != hipSuccess) return 3;
    CHECK(mr1l_destroy(plan));

    double* c_out = (double*)malloc((size_t)n * 16 + 1);
    double* y_out = (double*)malloc((size_t)sm * 16 + 1);
    if (!c_out || !y_out) return 3;
    if (hipMemcpy(c_out, dc, (size_t)n * 16, hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(y_out, dy_out, (size_t)sm * 16, hipMemcpyDeviceToHost) != hipSuccess)
        return 3;
    if (dump(dir, "coeffs_out", c_out, (size_t)n * 16) || dump(dir, "samples_out", y_out, (size_t)sm * 16)) return 4;
    printf("c_abi_example: n=%lld L=%d sum_M=%lld done (%s)\n", (long long)n, L, (long long)sm, mr1l_version());
    hipFree(dy);
    hipFree(dc);
    hipFree(dc_in);
    hipFree(dy_out);
    free(c_out);
    free(y_out);
    free(shape);
    free(freqs);
    free(M);
    free(z);
    free(samples);
    free(coeffs);
    return 0;
}
