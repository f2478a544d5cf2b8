/* A plain C consumer of libnqs: SR steps on the periodic TFIM chain N = 10,
 * J = h = 1, real RBM alpha = 1, 16 chains x 64 samples, 10 proposals between
 * samples, FP64; the caller allocates the workspace with hipMalloc.
 *
 * usage: vmc_chain <params.bin: P float64> <steps>
 * prints one line per step (energy mean, CG iterations), then the parameters. */
#include <stdio.h>
#include <stdlib.h>

#include <hip/hip_runtime_api.h>

#include "nqs.h"

#define CHECK(call)                                                              \
    do {                                                                         \
        int st_ = (call);                                                        \
        if (st_) {                                                               \
            fprintf(stderr, "%s: %d (%s)\n", #call, st_, nqs_last_error(ctx));  \
            return 1;                                                            \
        }                                                                        \
    } while (0)

int main(int argc, char** argv) {
    enum { N = 10 };
    nqs_ctx* ctx = NULL;
    int32_t bonds[2 * N];
    if (argc < 3) return 2;
    for (int i = 0; i < N; ++i) {
        bonds[2 * i] = i;
        bonds[2 * i + 1] = (i + 1) % N;
    }
    CHECK(nqs_create(&ctx, 0, NULL));
    CHECK(nqs_set_tfim(ctx, N, N, bonds, 1.0, 1.0));
    CHECK(nqs_set_rbm(ctx, N, 1, 1, NQS_FP64));
    CHECK(nqs_set_sampler(ctx, NQS_RULE_LOCAL, 16, 64, 10, 2, 0));
    const size_t ws = nqs_workspace_bytes(ctx);
    void* dev = NULL;
    if (hipMalloc(&dev, ws) != hipSuccess) return 3;
    CHECK(nqs_bind_workspace(ctx, dev, ws));
    const size_t P = nqs_num_params(ctx);
    double* p = (double*)malloc(P * sizeof(double));
    FILE* f = fopen(argv[1], "rb");
    if (!f || fread(p, sizeof(double), P, f) != P) return 4;
    fclose(f);
    CHECK(nqs_set_params(ctx, p, 0));
    const nqs_step_cfg cfg = {NQS_QGT_ONTHEFLY, 0.01, 0.02, 1e-10, 2000};
    const int steps = atoi(argv[2]);
    for (int k = 0; k < steps; ++k) {
        nqs_step_report rep;
        CHECK(nqs_vmc_step(ctx, &cfg, &rep));
        printf("%.17g %d\n", rep.energy.mean, rep.sr.iterations);
    }
    CHECK(nqs_get_params(ctx, p, 0));
    for (size_t k = 0; k < P; ++k) printf("%.17g\n", p[k]);
    nqs_destroy(ctx);
    hipFree(dev);
    free(p);
    return 0;
}
