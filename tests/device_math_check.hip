// Host-side check of the solver's device math (compiled for the host by a
// CPU test): the FP32 sin/cos of the circle map and the banded Cholesky.
//   sincos <amax> <count>   -> max |error| of sin and cos against libm
//   band                    -> reads "N B" then the packed lower triangle
//                              (B N (B N + 1) / 2 values, zeros outside the
//                              band) and the right-hand side; prints the
//                              factorisation flag, the solution and -g^T x
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>
#include "mpt_device.hpp"

template <int N, int B>
static int band_case()
{
    constexpr int M = B * N;
    double A[M * (M + 1) / 2], b[M];
    for (int i = 0; i < M * (M + 1) / 2; i++)
        if (scanf("%lf", &A[i]) != 1) return 1;
    for (int i = 0; i < M; i++)
        if (scanf("%lf", &b[i]) != 1) return 1;
    const bool ok = mpt::chol_band<double, N, B>(A);
    const double ysq = ok ? mpt::chol_solve_band<double, N, B>(A, b) : 0.0;
    printf("%d", ok ? 1 : 0);
    for (int i = 0; i < M; i++) printf(" %.17g", ok ? b[i] : 0.0);
    printf(" %.17g\n", ysq);
    return 0;
}

int main(int argc, char **argv)
{
    if (argc >= 4 && !strcmp(argv[1], "sincos")) {
        const double amax = atof(argv[2]);
        const long count = atol(argv[3]);
        double worst = 0.0;
        for (long i = 0; i <= count; i++) {
            const float a = (float)(-amax + 2.0 * amax * (double)i / (double)count);
            float s, c;
            mpt::sincos32(a, s, c);
            worst = fmax(worst, fabs((double)s - sin((double)a)));
            worst = fmax(worst, fabs((double)c - cos((double)a)));
        }
        printf("%.6e\n", worst);
        return 0;
    }
    if (argc >= 2 && !strcmp(argv[1], "band")) {
        int n, bw;
        while (scanf("%d %d", &n, &bw) == 2) {
            int r = 1;
#define CASE(NN, BB) if (n == NN && bw == BB) r = band_case<NN, BB>();
            CASE(1, 2) CASE(2, 2) CASE(3, 2) CASE(4, 2) CASE(5, 2)
            CASE(1, 3) CASE(2, 3) CASE(3, 3) CASE(4, 3) CASE(5, 3)
#undef CASE
            if (r) return r;
        }
        return 0;
    }
    fprintf(stderr, "usage: sincos <amax> <count> | band < cases\n");
    return 2;
}
