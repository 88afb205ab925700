// Batched Kalman filter for the moving obstacles (section "Kalman Filter",
// Eqs. 9-13): one thread per obstacle, FP64.
//
// State [x, y, vx, vy] (cells, cells per step), constant-velocity model with
// time step dt: A = [[I, dt I], [0, I]], B = 0, position measurement
// H = [I 0].  One call runs the time update x <- A x, P <- A P A^T + Q
// (Eqs. 9-10) and, when a measurement is given, the measurement update
// K = P H^T (H P H^T + R)^-1, x <- x + K (z - H x), P <- (I - K H) P
// (Eqs. 11-13), with the 2x2 inverse written out.  Matrix products are
// summed in index order, every product and sum rounded once (contraction is
// off for this file).
#include "twg_internal.h"

namespace twg {

namespace {

__global__ void k_kalman(int n, double *__restrict__ xs, double *__restrict__ Ps, const double *__restrict__ zs,
                         double dt, const double *__restrict__ Q, const double *__restrict__ R,
                         double *__restrict__ pos, double *__restrict__ vel)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double x[4], P[16];
    for (int k = 0; k < 4; ++k) x[k] = xs[4 * (size_t)i + k];
    for (int k = 0; k < 16; ++k) P[k] = Ps[16 * (size_t)i + k];
    const double A[16] = {1, 0, dt, 0, 0, 1, 0, dt, 0, 0, 1, 0, 0, 0, 0, 1};
    // time update
    double xn[4], AP[16], Pn[16];
    for (int r = 0; r < 4; ++r) {
        double acc = 0.0;
        for (int k = 0; k < 4; ++k) acc += A[r * 4 + k] * x[k];
        xn[r] = acc;
    }
    for (int r = 0; r < 4; ++r)
        for (int c = 0; c < 4; ++c) {
            double acc = 0.0;
            for (int k = 0; k < 4; ++k) acc += A[r * 4 + k] * P[k * 4 + c];
            AP[r * 4 + c] = acc;
        }
    for (int r = 0; r < 4; ++r)
        for (int c = 0; c < 4; ++c) {
            double acc = 0.0;
            for (int k = 0; k < 4; ++k) acc += AP[r * 4 + k] * A[c * 4 + k];
            Pn[r * 4 + c] = acc + (Q ? Q[r * 4 + c] : 0.0);
        }
    // measurement update
    if (zs) {
        const double z0 = zs[2 * (size_t)i], z1 = zs[2 * (size_t)i + 1];
        const double S0 = Pn[0] + R[0], S1 = Pn[1] + R[1], S2 = Pn[4] + R[2], S3 = Pn[5] + R[3];
        const double det = S0 * S3 - S1 * S2;
        const double Si0 = S3 / det, Si1 = -S1 / det, Si2 = -S2 / det, Si3 = S0 / det;
        double K[8];
        for (int r = 0; r < 4; ++r) {
            K[r * 2 + 0] = Pn[r * 4 + 0] * Si0 + Pn[r * 4 + 1] * Si2;
            K[r * 2 + 1] = Pn[r * 4 + 0] * Si1 + Pn[r * 4 + 1] * Si3;
        }
        const double in0 = z0 - xn[0], in1 = z1 - xn[1];
        for (int r = 0; r < 4; ++r) xn[r] = xn[r] + (K[r * 2 + 0] * in0 + K[r * 2 + 1] * in1);
        double Pu[16];
        for (int r = 0; r < 4; ++r)
            for (int c = 0; c < 4; ++c)
                Pu[r * 4 + c] = Pn[r * 4 + c] - (K[r * 2 + 0] * Pn[0 * 4 + c] + K[r * 2 + 1] * Pn[1 * 4 + c]);
        for (int k = 0; k < 16; ++k) Pn[k] = Pu[k];
    }
    for (int k = 0; k < 4; ++k) xs[4 * (size_t)i + k] = xn[k];
    for (int k = 0; k < 16; ++k) Ps[16 * (size_t)i + k] = Pn[k];
    if (pos) {
        pos[2 * (size_t)i] = xn[0];
        pos[2 * (size_t)i + 1] = xn[1];
    }
    if (vel) {
        vel[2 * (size_t)i] = xn[2];
        vel[2 * (size_t)i + 1] = xn[3];
    }
}

}  // namespace

int launch_kalman(int n, double *x, double *P, const double *z, double dt, const double *Q, const double *R,
                  double *pos, double *vel, hipStream_t st)
{
    if (n == 0) return TWG_OK;
    hipLaunchKernelGGL(k_kalman, dim3((n + 255) / 256), dim3(256), 0, st, n, x, P, z, dt, Q, R, pos, vel);
    return hipGetLastError() == hipSuccess ? TWG_OK : TWG_EDEVICE;
}

}  // namespace twg
