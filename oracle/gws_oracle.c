/*
 * FP64 dense CPU oracle for Gaussian Wave Splatting (fast, order-invariant variant).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or call this
 * file; it exists so that tests, the smoke check and the benchmark's CPU baseline can
 * compare the GPU library against a plain, slow, obviously correct evaluation of the
 * paper's formulas.  It shares no code, header, table or constant with the GPU path.
 *
 * Every quantity is evaluated directly from its definition in double precision:
 *   - the closed-form angular spectrum of an in-plane 2D Gaussian (Sec. 4.1, Eq. 9-10,
 *     with the 2D Fourier pair of Eq. 7 written in ordinary frequency: det J = 1 and
 *     det S = sqrt(det Sigma) for a Gaussian parallel to the SLM),
 *   - the angular-spectrum transfer function H (Eq. 3-4) evaluated at distance -z_i,
 *   - the order-invariant (approximated alpha wave blending) sum of Eq. 12, every
 *     Gaussian at every requested frequency, no culling,
 *   - for the adjoint: the analytic derivative of each term of Eq. 12 with respect to
 *     each Gaussian parameter, contracted with the spectrum-domain gradient.
 *
 * Conventions (the readings the paper leaves open; all pinned by tests):
 *   frequency nu is in cycles per metre; the forward transform kernel is exp(-j 2 pi nu.x),
 *   so a Gaussian centred at mu carries the ramp exp(-j 2 pi nu.mu);
 *   H(nu, d) = exp(+j 2 pi d sqrt(1/lambda^2 - |nu|^2)) for |nu| < 1/lambda, else 0;
 *   frequency index m maps to m' = m (m < N/2) or m - N (FFT order), nu = m' / (N p);
 *   the reference plane wave that illuminates every Gaussian (Sec. 4.1) has transverse
 *   frequency nu_r (cycles per metre, the same for every wavelength) and multiplies the
 *   Gaussian's own wavefront by exp(+j 2 pi nu_r.x) with x measured from the SLM centre, so
 *   the Gaussian's spectrum g_i is evaluated at nu - nu_r while H keeps the full nu.
 */
#include <math.h>
#include <stdint.h>

#define PI 3.14159265358979323846264338327950
#define TWO_PI (2.0 * PI)

static int signed_index(int m, int n) { return (m < n / 2) ? m : m - n; }

/*
 * Angular spectrum of the whole scene at a list of frequencies (Eq. 12):
 *   U_c(nu) = sum_i a_{c,i} o_i e^{j phi_i} g_i(nu - nu_r) H_c(nu, -z_i)
 *   g_i(nu) = 2 pi sqrt(det Sigma_i) exp(-2 pi^2 nu^T Sigma_i nu) exp(-j 2 pi nu.mu_i)   (Eq. 10)
 * Gaussians are summed in the order given.  amp is [n_lambda][n]; out is
 * [n_lambda][n_freq] interleaved (re, im).  The frequency list holds FFT-order indices.
 */
void oracle_spectrum(int64_t n, const double *mean_x, const double *mean_y, const double *depth,
                     const double *cov_xx, const double *cov_xy, const double *cov_yy,
                     const double *opacity, const double *amp, const double *phase,
                     int nx, int ny, double px, double py, int n_lambda, const double *lambdas,
                     double ref_nu_x, double ref_nu_y,
                     int64_t n_freq, const int32_t *freq_mx, const int32_t *freq_my, double *out)
{
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t f = 0; f < n_freq; ++f) {
        const double nu_x = signed_index(freq_mx[f], nx) / (nx * px);
        const double nu_y = signed_index(freq_my[f], ny) / (ny * py);
        const double nu2 = nu_x * nu_x + nu_y * nu_y;
        const double gx = nu_x - ref_nu_x, gy = nu_y - ref_nu_y;   /* argument of g_i */
        for (int c = 0; c < n_lambda; ++c) {
            const double inv_l = 1.0 / lambdas[c];
            double re = 0.0, im = 0.0;
            if (nu2 < inv_l * inv_l) {               /* evanescent band: H = 0 (Eq. 4) */
                const double kz = sqrt(inv_l * inv_l - nu2);   /* cycles per metre along z */
                for (int64_t i = 0; i < n; ++i) {
                    const double det = cov_xx[i] * cov_yy[i] - cov_xy[i] * cov_xy[i];
                    const double quad = gx * gx * cov_xx[i] + 2.0 * gx * gy * cov_xy[i]
                                      + gy * gy * cov_yy[i];
                    const double mag = amp[(int64_t)c * n + i] * opacity[i]
                                     * TWO_PI * sqrt(det) * exp(-2.0 * PI * PI * quad);
                    /* phase of e^{j phi} * ramp e^{-j 2 pi (nu - nu_r).mu} * H(nu, -z) */
                    const double ph = phase[i] - TWO_PI * (gx * mean_x[i] + gy * mean_y[i])
                                    + TWO_PI * (-depth[i]) * kz;
                    re += mag * cos(ph);
                    im += mag * sin(ph);
                }
            }
            out[2 * ((int64_t)c * n_freq + f)] = re;
            out[2 * ((int64_t)c * n_freq + f) + 1] = im;
        }
    }
}

/*
 * Gradient of a real loss L with respect to every parameter of the selected Gaussians,
 * given the spectrum-domain gradient gs = dL/dRe U + j dL/dIm U on the full grid
 * ([n_lambda][ny][nx] interleaved, FFT-order indices).  For a real parameter t,
 *   dL/dt = Re sum_{c,m} conj(gs_c(m)) * dU_c(m)/dt,
 * and each derivative of a term T of Eq. 12 is written out analytically, with
 * (g_x, g_y) = nu - nu_r the argument of the Gaussian's own spectrum:
 *   dT/dmu_x = -j 2 pi g_x T,  dT/dmu_y = -j 2 pi g_y T,  dT/dz = -j 2 pi kz T,
 *   dT/dphi  = j T,
 *   dT/dSxx = (Syy / (2 det) - 2 pi^2 g_x^2) T,  dT/dSyy = (Sxx / (2 det) - 2 pi^2 g_y^2) T,
 *   dT/dSxy = (-Sxy / det - 4 pi^2 g_x g_y) T  (Sxy is one parameter that fills both
 *            off-diagonal entries),
 *   dT/do   = a_c e^{j phi} g H,   dT/da_c = o e^{j phi} g H  (channel c only).
 * grad layout: [n_sel][9 + n_lambda] = mean_x, mean_y, depth, cov_xx, cov_xy, cov_yy,
 * opacity, phase, (unused 0), amplitude[c]...
 */
void oracle_param_grads(int64_t n, const double *mean_x, const double *mean_y, const double *depth,
                        const double *cov_xx, const double *cov_xy, const double *cov_yy,
                        const double *opacity, const double *amp, const double *phase,
                        int nx, int ny, double px, double py, int n_lambda, const double *lambdas,
                        double ref_nu_x, double ref_nu_y,
                        const double *gs, int64_t n_sel, const int64_t *sel, double *grad)
{
    const int stride = 9 + n_lambda;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t s = 0; s < n_sel; ++s) {
        const int64_t i = sel[s];
        const double det = cov_xx[i] * cov_yy[i] - cov_xy[i] * cov_xy[i];
        double g_mx = 0, g_my = 0, g_z = 0, g_sxx = 0, g_sxy = 0, g_syy = 0, g_o = 0, g_phi = 0;
        double g_a[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        for (int c = 0; c < n_lambda; ++c) {
            const double inv_l = 1.0 / lambdas[c];
            for (int my = 0; my < ny; ++my) {
                const double nu_y = signed_index(my, ny) / (ny * py);
                for (int mx = 0; mx < nx; ++mx) {
                    const double nu_x = signed_index(mx, nx) / (nx * px);
                    const double nu2 = nu_x * nu_x + nu_y * nu_y;
                    if (!(nu2 < inv_l * inv_l)) continue;
                    const double kz = sqrt(inv_l * inv_l - nu2);
                    const double gx = nu_x - ref_nu_x, gy = nu_y - ref_nu_y;
                    const double quad = gx * gx * cov_xx[i] + 2.0 * gx * gy * cov_xy[i]
                                      + gy * gy * cov_yy[i];
                    /* B = e^{j phi} g(nu - nu_r) H(nu,-z): the term without a_c and o */
                    const double bmag = TWO_PI * sqrt(det) * exp(-2.0 * PI * PI * quad);
                    const double ph = phase[i] - TWO_PI * (gx * mean_x[i] + gy * mean_y[i])
                                    + TWO_PI * (-depth[i]) * kz;
                    const double b_re = bmag * cos(ph), b_im = bmag * sin(ph);
                    const double ao = amp[(int64_t)c * n + i] * opacity[i];
                    const double t_re = ao * b_re, t_im = ao * b_im;
                    const int64_t k = ((int64_t)c * ny + my) * nx + mx;
                    const double q_re = gs[2 * k], q_im = gs[2 * k + 1];
                    /* Re(conj(q) * w) for w = x + j y is q_re x + q_im y */
#define RE_CONJ_Q(x, y) (q_re * (x) + q_im * (y))
                    /* (-j s) T = s (t_im, -t_re) */
                    g_mx += RE_CONJ_Q(TWO_PI * gx * t_im, -TWO_PI * gx * t_re);
                    g_my += RE_CONJ_Q(TWO_PI * gy * t_im, -TWO_PI * gy * t_re);
                    g_z += RE_CONJ_Q(TWO_PI * kz * t_im, -TWO_PI * kz * t_re);
                    const double wxx = cov_yy[i] / (2.0 * det) - 2.0 * PI * PI * gx * gx;
                    const double wyy = cov_xx[i] / (2.0 * det) - 2.0 * PI * PI * gy * gy;
                    const double wxy = -cov_xy[i] / det - 4.0 * PI * PI * gx * gy;
                    g_sxx += wxx * RE_CONJ_Q(t_re, t_im);
                    g_syy += wyy * RE_CONJ_Q(t_re, t_im);
                    g_sxy += wxy * RE_CONJ_Q(t_re, t_im);
                    g_phi += RE_CONJ_Q(-t_im, t_re);          /* j T = (-t_im, t_re) */
                    g_o += amp[(int64_t)c * n + i] * RE_CONJ_Q(b_re, b_im);
                    g_a[c] += opacity[i] * RE_CONJ_Q(b_re, b_im);
#undef RE_CONJ_Q
                }
            }
        }
        double *gr = grad + s * stride;
        gr[0] = g_mx; gr[1] = g_my; gr[2] = g_z; gr[3] = g_sxx; gr[4] = g_sxy; gr[5] = g_syy;
        gr[6] = g_o; gr[7] = g_phi; gr[8] = 0.0;
        for (int c = 0; c < n_lambda; ++c) gr[9 + c] = g_a[c];
    }
}
