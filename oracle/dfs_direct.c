/*
 * ORACLE -- test infrastructure only.  Nothing in the product path links,
 * loads or calls this file; only the tests, the smoke check and the CPU
 * baseline leg of the benchmark do.
 *
 * Plain FP64 evaluation of the bivariate complex-exponential DFS series
 * (section 5, eq. std_dfs_exp):
 *
 *     f(phi, theta) = sum_{n=-N..N} sum_{m=-M..M} ft[n,m] e^{i m phi} e^{i n theta}
 *
 * directly at every point, i.e. the O((M_lon N_lat)^2) route that the paper
 * names as the cost the NUFFT avoids.  There is no FFT, no kernel, no
 * wrapping: the exponentials are 2 pi periodic, so any real coordinate is
 * evaluated as given.
 *
 * Layout: coeffs is [n_fields][K_theta][K_phi] complex (re, im interleaved),
 * centred indices: row a <-> n = a - K_theta/2, column b <-> m = b - K_phi/2.
 * out is [n_fields][n_pts] complex.
 *
 * Per point the phase factors e^{i m phi} and e^{i n theta} are taken from
 * libm cos/sin of the FP64 product m*phi (no recurrence), then the sum is
 * done as row sums over m (ascending) followed by the sum over n
 * (ascending).  That grouping is the definition with the two sums nested
 * in the order the equation writes them; fields share the phase factors.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

#ifdef _OPENMP
#include <omp.h>
#endif

int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void oracle_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* Returns 0 on success, -1 on bad arguments or allocation failure. */
int oracle_dfs_eval(const double *coeffs, int64_t K_theta, int64_t K_phi,
                    int32_t n_fields, const double *phi, const double *theta,
                    int64_t n_pts, double *out)
{
    if (!coeffs || !phi || !theta || !out || K_theta <= 0 || K_phi <= 0 ||
        n_fields <= 0 || n_pts < 0)
        return -1;
    const int64_t n0 = K_theta / 2, m0 = K_phi / 2;
    int failed = 0;

#pragma omp parallel
    {
        double *ep = (double *)malloc(sizeof(double) * 2 * (size_t)K_phi);
        double *et = (double *)malloc(sizeof(double) * 2 * (size_t)K_theta);
        if (!ep || !et) {
#pragma omp atomic write
            failed = 1;
        }
#pragma omp for schedule(dynamic, 16)
        for (int64_t j = 0; j < n_pts; ++j) {
            if (!ep || !et) continue;
            const double ph = phi[j], th = theta[j];
            for (int64_t b = 0; b < K_phi; ++b) {
                const double arg = (double)(b - m0) * ph;
                ep[2 * b] = cos(arg);
                ep[2 * b + 1] = sin(arg);
            }
            for (int64_t a = 0; a < K_theta; ++a) {
                const double arg = (double)(a - n0) * th;
                et[2 * a] = cos(arg);
                et[2 * a + 1] = sin(arg);
            }
            for (int32_t f = 0; f < n_fields; ++f) {
                const double *Ff = coeffs + (size_t)2 * f * K_theta * K_phi;
                double cr = 0.0, ci = 0.0;
                for (int64_t a = 0; a < K_theta; ++a) {
                    const double *row = Ff + (size_t)2 * a * K_phi;
                    double rr = 0.0, ri = 0.0;
                    for (int64_t b = 0; b < K_phi; ++b) {
                        const double fr = row[2 * b], fi = row[2 * b + 1];
                        rr += fr * ep[2 * b] - fi * ep[2 * b + 1];
                        ri += fr * ep[2 * b + 1] + fi * ep[2 * b];
                    }
                    cr += rr * et[2 * a] - ri * et[2 * a + 1];
                    ci += rr * et[2 * a + 1] + ri * et[2 * a];
                }
                out[2 * ((size_t)f * n_pts + j)] = cr;
                out[2 * ((size_t)f * n_pts + j) + 1] = ci;
            }
        }
        free(ep);
        free(et);
    }
    return failed ? -1 : 0;
}

/*
 * The same sum carried in long double (x87 extended precision) with long
 * double cosl/sinl.  Used only to certify the FP64 oracle's own rounding on
 * a handful of points at the largest mode counts.
 */
int oracle_dfs_eval_ld(const double *coeffs, int64_t K_theta, int64_t K_phi,
                       int32_t n_fields, const double *phi, const double *theta,
                       int64_t n_pts, double *out)
{
    if (!coeffs || !phi || !theta || !out || K_theta <= 0 || K_phi <= 0 ||
        n_fields <= 0 || n_pts < 0)
        return -1;
    const int64_t n0 = K_theta / 2, m0 = K_phi / 2;
    int failed = 0;

#pragma omp parallel
    {
        long double *ep = (long double *)malloc(sizeof(long double) * 2 * (size_t)K_phi);
        long double *et = (long double *)malloc(sizeof(long double) * 2 * (size_t)K_theta);
        if (!ep || !et) {
#pragma omp atomic write
            failed = 1;
        }
#pragma omp for schedule(dynamic, 1)
        for (int64_t j = 0; j < n_pts; ++j) {
            if (!ep || !et) continue;
            const long double ph = phi[j], th = theta[j];
            for (int64_t b = 0; b < K_phi; ++b) {
                const long double arg = (long double)(b - m0) * ph;
                ep[2 * b] = cosl(arg);
                ep[2 * b + 1] = sinl(arg);
            }
            for (int64_t a = 0; a < K_theta; ++a) {
                const long double arg = (long double)(a - n0) * th;
                et[2 * a] = cosl(arg);
                et[2 * a + 1] = sinl(arg);
            }
            for (int32_t f = 0; f < n_fields; ++f) {
                const double *Ff = coeffs + (size_t)2 * f * K_theta * K_phi;
                long double cr = 0.0L, ci = 0.0L;
                for (int64_t a = 0; a < K_theta; ++a) {
                    const double *row = Ff + (size_t)2 * a * K_phi;
                    long double rr = 0.0L, ri = 0.0L;
                    for (int64_t b = 0; b < K_phi; ++b) {
                        const long double fr = row[2 * b], fi = row[2 * b + 1];
                        rr += fr * ep[2 * b] - fi * ep[2 * b + 1];
                        ri += fr * ep[2 * b + 1] + fi * ep[2 * b];
                    }
                    cr += rr * et[2 * a] - ri * et[2 * a + 1];
                    ci += rr * et[2 * a + 1] + ri * et[2 * a];
                }
                out[2 * ((size_t)f * n_pts + j)] = (double)cr;
                out[2 * ((size_t)f * n_pts + j) + 1] = (double)ci;
            }
        }
        free(ep);
        free(et);
    }
    return failed ? -1 : 0;
}
