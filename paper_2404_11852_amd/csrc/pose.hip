// Host-side camera pose arithmetic of the reference schedule: Eq. 5-6
// extrapolation and Eq. 2's relative transform.  float64 throughout, each
// result rounded once to float32.  No device work.
#include <cmath>

#include "cicero.h"

namespace {

struct Pose {
    double R[3][3];
    double c[3];
};

bool load(const float p[12], Pose &o)
{
    for (int i = 0; i < 12; ++i)
        if (!std::isfinite(p[i])) return false;
    for (int r = 0; r < 3; ++r) {
        for (int k = 0; k < 3; ++k) o.R[r][k] = (double)p[4 * r + k];
        o.c[r] = (double)p[4 * r + 3];
    }
    return true;
}

void store(const double R[3][3], const double c[3], float out[12])
{
    for (int r = 0; r < 3; ++r) {
        for (int k = 0; k < 3; ++k) out[4 * r + k] = (float)R[r][k];
        out[4 * r + 3] = (float)c[r];
    }
}

// C = A B
void matmul(const double A[3][3], const double B[3][3], double C[3][3])
{
    for (int r = 0; r < 3; ++r)
        for (int k = 0; k < 3; ++k) C[r][k] = A[r][0] * B[0][k] + A[r][1] * B[1][k] + A[r][2] * B[2][k];
}

// C = A B^T
void matmul_bt(const double A[3][3], const double B[3][3], double C[3][3])
{
    for (int r = 0; r < 3; ++r)
        for (int k = 0; k < 3; ++k) C[r][k] = A[r][0] * B[k][0] + A[r][1] * B[k][1] + A[r][2] * B[k][2];
}

// Rotation by angle phi about the unit axis a (Rodrigues).
void axis_angle(const double a[3], double phi, double M[3][3])
{
    const double s = std::sin(phi), v = 1.0 - std::cos(phi);
    const double K[3][3] = {{0.0, -a[2], a[1]}, {a[2], 0.0, -a[0]}, {-a[1], a[0], 0.0}};
    double K2[3][3];
    matmul(K, K, K2);
    for (int r = 0; r < 3; ++r)
        for (int k = 0; k < 3; ++k) M[r][k] = (r == k ? 1.0 : 0.0) + s * K[r][k] + v * K2[r][k];
}

// Q^steps for a rotation matrix Q, through its axis-angle form.
void rotation_power(const double Q[3][3], double steps, double M[3][3])
{
    const double w[3] = {Q[2][1] - Q[1][2], Q[0][2] - Q[2][0], Q[1][0] - Q[0][1]};   // 2 sin(theta) axis
    const double sn = std::sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
    const double cs = Q[0][0] + Q[1][1] + Q[2][2] - 1.0;                              // 2 cos(theta)
    const double theta = std::atan2(sn, cs);
    double a[3];
    if (sn > 1e-9) {
        for (int k = 0; k < 3; ++k) a[k] = w[k] / sn;
    } else if (cs > 0.0) {
        for (int r = 0; r < 3; ++r)
            for (int k = 0; k < 3; ++k) M[r][k] = r == k ? 1.0 : 0.0;
        return;
    } else {
        // half turn: (Q + I)/2 = a a^T; take the column with the largest diagonal
        int j = 0;
        for (int k = 1; k < 3; ++k)
            if (Q[k][k] > Q[j][j]) j = k;
        const double d = std::sqrt(0.5 * (Q[j][j] + 1.0));
        for (int k = 0; k < 3; ++k) a[k] = (k == j) ? d : 0.5 * Q[k][j] / d;
        const double n = std::sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]);
        for (int k = 0; k < 3; ++k) a[k] /= n;
    }
    axis_angle(a, steps * theta, M);
}

}  // namespace

extern "C" {

int cic_extrapolate_pose(const float c2w_prev[12], const float c2w_cur[12], float steps, float c2w_out[12])
{
    Pose p, q;
    if (!c2w_prev || !c2w_cur || !c2w_out || !std::isfinite(steps)) return CIC_ERR_INVALID;
    if (!load(c2w_prev, p) || !load(c2w_cur, q)) return CIC_ERR_INVALID;
    const double s = (double)steps;
    double c[3];
    for (int k = 0; k < 3; ++k) c[k] = q.c[k] + s * (q.c[k] - p.c[k]);
    double Q[3][3], M[3][3], R[3][3];
    matmul_bt(q.R, p.R, Q);       // world-frame rotation from the older orientation to the newer one
    rotation_power(Q, s, M);
    matmul(M, q.R, R);
    store(R, c, c2w_out);
    return CIC_OK;
}

int cic_relative_pose(const float c2w_ref[12], const float c2w_tgt[12], float ref_T_tgt[12])
{
    Pose a, b;
    if (!c2w_ref || !c2w_tgt || !ref_T_tgt) return CIC_ERR_INVALID;
    if (!load(c2w_ref, a) || !load(c2w_tgt, b)) return CIC_ERR_INVALID;
    double R[3][3], t[3];
    for (int r = 0; r < 3; ++r) {
        for (int k = 0; k < 3; ++k) R[r][k] = b.R[0][r] * a.R[0][k] + b.R[1][r] * a.R[1][k] + b.R[2][r] * a.R[2][k];
        t[r] = b.R[0][r] * (a.c[0] - b.c[0]) + b.R[1][r] * (a.c[1] - b.c[1]) + b.R[2][r] * (a.c[2] - b.c[2]);
    }
    store(R, t, ref_T_tgt);
    return CIC_OK;
}

}  // extern "C"
