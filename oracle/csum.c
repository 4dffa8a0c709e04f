/*
 * Plain all-pairs Green's function sum for the oracle (test infrastructure).
 *
 * U[a][k] = sum over source patches j != tgt[a], sum over skeleton points m of
 *           G(|Z[tgt[a]][k] - S[j][m]|) * rho[j][m]
 *
 * G is the sphere's on-surface Neumann Green's function (paper Section 2.1):
 *   exterior (problem 1): 2/d - log(2/d) - log(1 + d/2)
 *   interior (problem 0): 2/d + log(2/d) - log(1 + d/2)
 *
 * Z: N x nz x 3 target points, S: N x ns x 3 source points, rho: N x ns,
 * tgt: ntgt target patch indices, U: ntgt x nz output. FP64, no reordering
 * of the definition; OpenMP over target points only.
 */
#include <math.h>

static double g_surface(double d, int problem)
{
    if (problem == 1)
        return 2.0 / d - log(2.0 / d) - log1p(0.5 * d);
    return 2.0 / d + log(2.0 / d) - log1p(0.5 * d);
}

void nce_oracle_incoming(int problem, long N, long nz, const double *Z, long ns,
                         const double *S, const double *rho, long ntgt,
                         const long *tgt, double *U)
{
    long total = ntgt * nz;
#pragma omp parallel for schedule(dynamic, 16)
    for (long q = 0; q < total; ++q) {
        long a = q / nz, k = q % nz;
        long i = tgt[a];
        const double *z = Z + (i * nz + k) * 3;
        double acc = 0.0;
        for (long j = 0; j < N; ++j) {
            if (j == i)
                continue;
            const double *s = S + j * ns * 3;
            const double *r = rho + j * ns;
            for (long m = 0; m < ns; ++m) {
                double dx = z[0] - s[3 * m], dy = z[1] - s[3 * m + 1], dz = z[2] - s[3 * m + 2];
                double d = sqrt(dx * dx + dy * dy + dz * dz);
                acc += g_surface(d, problem) * r[m];
            }
        }
        U[q] = acc;
    }
}
