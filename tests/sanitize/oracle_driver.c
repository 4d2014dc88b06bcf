/* Drives the oracle's entry points on small inputs; built with AddressSanitizer
 * and UndefinedBehaviorSanitizer by tests/test_sanitizers.py (test
 * infrastructure: it exercises the oracle's memory accesses, not its values). */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int orc_heat(int d, const int64_t* N, int64_t nplanes, double tau, const double* in, double* out, int naive,
             double* max_imag);
int orc_project(int64_t npts, int n, const double* A, double* Q, int8_t* detsign, double* sigma, int32_t* sweeps);
int orc_iterate(int d, const int64_t* N, int n, double tau, double* A, int K, double tol, int* iters,
                double* energy, int64_t* flips, double* delta, double* max_imag, int naive);
int orc_project_vjp(int64_t npts, int n, const double* A, const double* G, double* GA);
int orc_unroll_grad(int d, const int64_t* N, int n, double tau, const double* A0, const double* T, int K,
                    double* loss, double* gA0, double* gtau, int64_t* flips);
int orc_volume_project(int64_t npts, int n, const double* A, int64_t n_plus, double* B, double* dE, int8_t* sel);

static double urand(uint64_t* s)
{
    *s = *s * 6364136223846793005ull + 1442695040888963407ull;
    return (double)(*s >> 11) / 9007199254740992.0 * 2.0 - 1.0;
}

int main(void)
{
    uint64_t seed = 12345;
    const int64_t N2[2] = {8, 16}, N3[3] = {8, 4, 8};
    int rc = 0;
    for (int n = 1; n <= 4; ++n) {
        for (int d = 2; d <= 3; ++d) {
            const int64_t* N = d == 2 ? N2 : N3;
            int64_t P = 1;
            for (int a = 0; a < d; ++a) P *= N[a];
            const int64_t E = (int64_t)n * n * P;
            double *A = malloc(sizeof(double) * E), *B = malloc(sizeof(double) * E), *G = malloc(sizeof(double) * E);
            double *H = malloc(sizeof(double) * E), *sg = malloc(sizeof(double) * n * P), *dE = malloc(sizeof(double) * P);
            int8_t *ds = malloc(P), *sel = malloc(P);
            int32_t* sw = malloc(sizeof(int32_t) * P);
            for (int64_t i = 0; i < E; ++i) { A[i] = urand(&seed); G[i] = urand(&seed); }
            double mi = 0, en[4], dl[3], loss, gtau;
            int64_t fl[3];
            int it = 0;
            rc |= orc_heat(d, N, (int64_t)n * n, 1e-3, A, H, 0, &mi);
            rc |= orc_heat(d, N, (int64_t)n * n, 1e-3, A, H, 1, &mi);
            rc |= orc_project(P, n, A, B, ds, sg, sw);
            rc |= orc_project_vjp(P, n, A, G, H);
            for (int64_t i = 0; i < E; ++i) B[i] = A[i];
            rc |= orc_iterate(d, N, n, 2e-3, B, 3, 1e-300, &it, en, fl, dl, &mi, 0);
            rc |= orc_unroll_grad(d, N, n, 2e-3, A, G, 3, &loss, H, &gtau, fl);
            if (n >= 2) rc |= orc_volume_project(P, n, A, P / 2, B, dE, sel);
            free(A); free(B); free(G); free(H); free(sg); free(dE); free(ds); free(sel); free(sw);
        }
    }
    printf("oracle driver done rc=%d\n", rc);
    return rc != 0;
}
