// Internal host-side interface between the C ABI and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lagp {

constexpr int kMaxP = 16;  // largest input dimension any kernel accepts

struct AlcArgs {
    const double *X;
    const double *Y;
    int64_t N;
    int p;
    const double *XX;
    int64_t M;
    const int32_t *pool;
    int Np;
    int n0;
    int n;
    double d;
    double g;
    double *mean;
    double *s2;
    double *var;
    int32_t *sel;
    double *alc;
    int32_t *status;
    int32_t *guard;
};

// Largest LDS buffer the NN kernel needs for a pool of Np (0 if unsupported).
int nn_pool_cap(int Np);
hipError_t launch_nn_pool(const double *X, int64_t N, int p, const double *XX, int64_t M, int Np,
                          int32_t *pool, hipStream_t st);

// Returns hipErrorNotSupported (without launching) when no compiled schedule
// covers (p, Np, n, precision).
bool alc_supported(int precision, int p, int Np, int n);
hipError_t launch_alc(const AlcArgs &a, int precision, hipStream_t st);

}  // namespace lagp
