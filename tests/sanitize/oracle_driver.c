/* Host driver for the sanitizer build of the C oracle (oracle/gws_oracle.c): the spectrum at
 * every frequency of a small odd-sized grid and the gradients of a few selected Gaussians,
 * with two wavelengths and an off-axis reference wave, so every loop and index of both entry
 * points runs.  Prints OK and exits 0 when every output is finite. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

void oracle_spectrum(int64_t n, const double *mean_x, const double *mean_y, const double *depth,
                     const double *cov_xx, const double *cov_xy, const double *cov_yy,
                     const double *opacity, const double *amp, const double *phase,
                     int nx, int ny, double px, double py, int n_lambda, const double *lambdas,
                     double ref_nu_x, double ref_nu_y,
                     int64_t n_freq, const int32_t *freq_mx, const int32_t *freq_my, double *out);
void oracle_param_grads(int64_t n, const double *mean_x, const double *mean_y, const double *depth,
                        const double *cov_xx, const double *cov_xy, const double *cov_yy,
                        const double *opacity, const double *amp, const double *phase,
                        int nx, int ny, double px, double py, int n_lambda, const double *lambdas,
                        double ref_nu_x, double ref_nu_y,
                        const double *gs, int64_t n_sel, const int64_t *sel, double *grad);

int main(void)
{
    enum { N = 5, NX = 21, NY = 18, C = 2 };
    const double px = 8e-6, py = 8e-6, lambdas[C] = {520e-9, 638e-9};
    double mx[N], my[N], z[N], sxx[N], sxy[N], syy[N], o[N], a[C * N], ph[N];
    for (int i = 0; i < N; ++i) {
        mx[i] = (i - 2) * 9e-6;
        my[i] = (2 - i) * 7e-6;
        z[i] = (i - 2) * 1e-3;
        sxx[i] = (2.0 + i) * 1e-11;
        sxy[i] = 0.3e-11;
        syy[i] = (3.0 + 0.5 * i) * 1e-11;
        o[i] = 0.2 + 0.15 * i;
        ph[i] = 0.7 * i;
        for (int c = 0; c < C; ++c) a[c * N + i] = 0.5 + 0.1 * c + 0.05 * i;
    }
    int32_t fmx[NX * NY], fmy[NX * NY];
    for (int y = 0; y < NY; ++y)
        for (int x = 0; x < NX; ++x) {
            fmx[y * NX + x] = x;
            fmy[y * NX + x] = y;
        }
    double *spec = malloc(sizeof(double) * 2 * C * NX * NY);
    oracle_spectrum(N, mx, my, z, sxx, sxy, syy, o, a, ph, NX, NY, px, py, C, lambdas, 1234.5, -321.0, NX * NY,
                    fmx, fmy, spec);
    int bad = 0;
    for (int k = 0; k < 2 * C * NX * NY; ++k) bad |= !isfinite(spec[k]);
    int64_t sel[3] = {0, 2, 4};
    double *grad = malloc(sizeof(double) * 3 * (9 + C));
    oracle_param_grads(N, mx, my, z, sxx, sxy, syy, o, a, ph, NX, NY, px, py, C, lambdas, 1234.5, -321.0, spec, 3,
                       sel, grad);
    for (int k = 0; k < 3 * (9 + C); ++k) bad |= !isfinite(grad[k]);
    free(spec);
    free(grad);
    printf("%s\n", bad ? "FAIL" : "OK");
    return bad;
}
