// Holographics transform (supplement, Holographics pipeline; Sec. 4 view-dependent opacity):
// world-space Gaussians and a camera to the in-plane hologram-space Gaussians the splatting
// kernels take.  One thread per Gaussian; the arithmetic is FP64 (the kernel moves ~130 bytes
// per Gaussian and does a few hundred flops, so it is bound by HBM either way) and the
// outputs are rounded to FP32 once.
//
//   model:      Sigma_w = R_w S_w S_w^T R_w^T, R_w from the quaternion (w, x, y, z), S_w = diag(s)
//   view:       p = R_v mu_w + t (the camera looks along -z)
//   projection: Pi(p) = (f_x p_x / -p_z + c_x, f_y p_y / -p_z + c_y), J = dPi/dp at p,
//               Sigma_r = J R_v Sigma_w R_v^T J^T (EWA local affine approximation)
//   lift:       depth p_z, zero z-scale, no rotation about x or y
//   hologram:   in-plane 2 x 2 map A plus offset, depth z_h = a p_z + b
//   opacity:    sum_k o_k Y_k(d), d = (mu_w - camera centre) / |...|, clamped to [0, 1];
//               real spherical harmonics with the Condon-Shortley phase, k = l^2 + l + m
// Gaussians closer than `near` in front of the camera get opacity 0 and a zero covariance
// (the splatting kernels cull both).
#include "gws_internal.h"

namespace gws {

// Real spherical harmonics of the unit vector (x, y, z), degree <= 3, into y[0 .. 15].
static __device__ __forceinline__ void real_sh3(double x, double y, double z, double *Y)
{
    const double xx = x * x, yy = y * y, zz = z * z;
    Y[0] = 0.28209479177387814;                           // 1 / (2 sqrt(pi))
    const double c1 = 0.48860251190291992;                // sqrt(3 / (4 pi))
    Y[1] = -c1 * y;
    Y[2] = c1 * z;
    Y[3] = -c1 * x;
    const double c2a = 1.0925484305920792;                // sqrt(15 / pi) / 2
    const double c2b = 0.31539156525252005;               // sqrt(5 / pi) / 4
    const double c2c = 0.54627421529603959;               // sqrt(15 / pi) / 4
    Y[4] = c2a * x * y;
    Y[5] = -c2a * y * z;
    Y[6] = c2b * (2.0 * zz - xx - yy);
    Y[7] = -c2a * x * z;
    Y[8] = c2c * (xx - yy);
    const double c3a = 0.59004358992664352;               // sqrt(35 / (2 pi)) / 4
    const double c3b = 2.8906114426405538;                // sqrt(105 / pi) / 2
    const double c3c = 0.45704579946446572;               // sqrt(21 / (2 pi)) / 4
    const double c3d = 0.37317633259011540;               // sqrt(7 / pi) / 4
    const double c3e = 1.4453057213202769;                // sqrt(105 / pi) / 4
    Y[9] = -c3a * y * (3.0 * xx - yy);
    Y[10] = c3b * x * y * z;
    Y[11] = -c3c * y * (4.0 * zz - xx - yy);
    Y[12] = c3d * z * (2.0 * zz - 3.0 * xx - 3.0 * yy);
    Y[13] = -c3c * x * (4.0 * zz - xx - yy);
    Y[14] = c3e * z * (xx - yy);
    Y[15] = -c3a * x * (xx - 3.0 * yy);
}

__global__ void __launch_bounds__(256) k_holographics(HoloArgs a, int64_t n, const float *__restrict__ mean,
                                                      const float *__restrict__ quat, const float *__restrict__ scale,
                                                      const float *__restrict__ sh, PlaneOut out)
{
    const int K = (a.sh_degree + 1) * (a.sh_degree + 1);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const double mw[3] = {mean[3 * i], mean[3 * i + 1], mean[3 * i + 2]};
        // view space
        double p[3];
        for (int r = 0; r < 3; ++r) p[r] = a.R[3 * r] * mw[0] + a.R[3 * r + 1] * mw[1] + a.R[3 * r + 2] * mw[2] + a.t[r];
        if (!(-p[2] >= a.near)) {
            out.mean_x[i] = out.mean_y[i] = out.depth[i] = 0.0f;
            out.cov_xx[i] = out.cov_xy[i] = out.cov_yy[i] = 0.0f;
            out.opacity[i] = 0.0f;
            continue;
        }
        // model transform M = R_w diag(s)
        double qw = quat[4 * i], qx = quat[4 * i + 1], qy = quat[4 * i + 2], qz = quat[4 * i + 3];
        const double qn = sqrt(qw * qw + qx * qx + qy * qy + qz * qz);
        const double iq = qn > 0.0 ? 1.0 / qn : 0.0;
        qw = qn > 0.0 ? qw * iq : 1.0;
        qx *= iq;
        qy *= iq;
        qz *= iq;
        const double Rw[9] = {1 - 2 * (qy * qy + qz * qz), 2 * (qx * qy - qw * qz), 2 * (qx * qz + qw * qy),
                              2 * (qx * qy + qw * qz), 1 - 2 * (qx * qx + qz * qz), 2 * (qy * qz - qw * qx),
                              2 * (qx * qz - qw * qy), 2 * (qy * qz + qw * qx), 1 - 2 * (qx * qx + qy * qy)};
        const double s[3] = {scale[3 * i], scale[3 * i + 1], scale[3 * i + 2]};
        // B = R_v R_w diag(s) (3 x 3)
        double B[9];
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c)
                B[3 * r + c] = (a.R[3 * r] * Rw[c] + a.R[3 * r + 1] * Rw[3 + c] + a.R[3 * r + 2] * Rw[6 + c]) * s[c];
        // projection and its Jacobian at p
        const double iz = 1.0 / -p[2];
        const double u = a.fx * p[0] * iz + a.cx, v = a.fy * p[1] * iz + a.cy;
        const double J0[3] = {a.fx * iz, 0.0, a.fx * p[0] * iz * iz};
        const double J1[3] = {0.0, a.fy * iz, a.fy * p[1] * iz * iz};
        // G = A J B (2 x 3): hologram-space factor of the covariance, Sigma_h = G G^T
        double JB0[3], JB1[3];
        for (int c = 0; c < 3; ++c) {
            JB0[c] = J0[0] * B[c] + J0[1] * B[3 + c] + J0[2] * B[6 + c];
            JB1[c] = J1[0] * B[c] + J1[1] * B[3 + c] + J1[2] * B[6 + c];
        }
        double G0[3], G1[3];
        for (int c = 0; c < 3; ++c) {
            G0[c] = a.A[0] * JB0[c] + a.A[1] * JB1[c];
            G1[c] = a.A[2] * JB0[c] + a.A[3] * JB1[c];
        }
        out.cov_xx[i] = (float)(G0[0] * G0[0] + G0[1] * G0[1] + G0[2] * G0[2]);
        out.cov_xy[i] = (float)(G0[0] * G1[0] + G0[1] * G1[1] + G0[2] * G1[2]);
        out.cov_yy[i] = (float)(G1[0] * G1[0] + G1[1] * G1[1] + G1[2] * G1[2]);
        out.mean_x[i] = (float)(a.A[0] * u + a.A[1] * v + a.b[0]);
        out.mean_y[i] = (float)(a.A[2] * u + a.A[3] * v + a.b[1]);
        out.depth[i] = (float)(a.depth_scale * p[2] + a.depth_offset);
        // view-dependent opacity
        const double dx = mw[0] - a.centre[0], dy = mw[1] - a.centre[1], dz = mw[2] - a.centre[2];
        const double dn = sqrt(dx * dx + dy * dy + dz * dz);
        const double id = dn > 0.0 ? 1.0 / dn : 0.0;
        double Y[16];
        real_sh3(dx * id, dy * id, dz * id, Y);
        double o = 0.0;
        for (int k = 0; k < K; ++k) o += (double)sh[(int64_t)K * i + k] * Y[k];
        out.opacity[i] = (float)fmin(fmax(o, 0.0), 1.0);
    }
}

hipError_t launch_holographics(const HoloArgs &a, int64_t n, const float *mean, const float *quat, const float *scale,
                               const float *sh, const PlaneOut &out, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    const int64_t want = (n + 255) / 256;
    const int nb = (int)(want < 65536 ? want : 65536);
    hipLaunchKernelGGL(k_holographics, dim3(nb), dim3(256), 0, s, a, n, mean, quat, scale, sh, out);
    return hipGetLastError();
}

}  // namespace gws
