// ts_device.h -- device-side definitions shared by the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "ts.h"

namespace ts {

constexpr int kTile = TS_TILE;
constexpr int kBlock = 256;          // threads per tile workgroup (4 wave64)
constexpr int kWave = 64;

// Raster record of one visible triangle, 128 bytes (one L2 line).
//
// The window of Eq. (1) is rewritten as three affine functions of the
// pixel: with lambda_k the barycentric coordinate of the vertex opposite
// edge k, P the perimeter and l_k the edge length,
//     phi(p)/phi(s) = min_k lambda_k(p) P / l_k = min_k u_k(p),
// because the distance from p to edge k is lambda_k(p) times the height on
// that edge (2A/l_k) and phi(s) = -r = -2A/P.  The u_k coefficients are
// stored in FP64 relative to an integer anchor pixel (ax, ay) so that
// u_k(p) = A_k dx + B_k dy + C_k with dx = px - ax, dy = py - ay exact
// integers (the pixel centre's 1/2 is folded into C_k).
//
// The two alternative windows store the distance form instead: u_k(p) is
// the signed distance from p to edge k (positive inside), the above times
// the inradius r.
//
// Byte layout (16-byte chunks): 0-3 A, B, C[0..1]; 4 C[2], anchor, o;
// 5 sigma, rgb; 6 z, tight box, index; 7 ut, phis.  The rasterizers stage
// chunks 0-5 and z in LDS (and phis for the LogSumExp window).
struct alignas(16) TriRecord {
    double A[3];
    double B[3];
    double C[3];
    int16_t ax, ay;              // anchor pixel
    float o;
    float sigma;
    float rgb[3];
    float z;
    int16_t px0, px1, py0, py1;  // tight pixel box
    uint32_t tri;
    float ut;     // lower bound of u over the pixels that can composite: u_min (1 - 2^-10)
    float phis;   // LogSumExp window: phi_lse(s) = ln 3 - r (< 0); else 0
    float pad[2];
};
static_assert(sizeof(TriRecord) == 128, "record must be one 128-byte line");
static_assert(offsetof(TriRecord, o) == 76 && offsetof(TriRecord, sigma) == 80 &&
                  offsetof(TriRecord, z) == 96 && offsetof(TriRecord, ut) == 112 &&
                  offsetof(TriRecord, phis) == 116,
              "chunk layout the rasterizers stage");

constexpr double kLn3 = 1.0986122886681098;   // ln 3

struct Cam {
    float R[9], t[3], fx, fy, cx, cy;
    int W, H;
};

struct Cfg {
    float alpha_min, alpha_max, T_min, z_near, r_min;
    int deg;
    float bg[3];
    int window;   // TS_WINDOW_*
};

// ---------------------------------------------------------------------------
// Real orthonormal SH up to degree 3 in Cartesian form (unit direction
// x, y, z), index l*l + l + m, no Condon-Shortley phase:
//   Y_l^0 = N_l^0 P_l(z),  Y_l^{+-m} = sqrt(2) N_l^m {Re, Im}(x+iy)^m P_l^(m)(z)
// expanded by hand; the constants are the products of the normalisations.
// ---------------------------------------------------------------------------
namespace shc {
constexpr float c0 = 0.28209479177387814f;   // 1/(2 sqrt(pi))
constexpr float c1 = 0.48860251190291992f;   // sqrt(3/(4pi))
constexpr float c2a = 1.0925484305920792f;   // sqrt(15/(4pi))
constexpr float c2b = 0.31539156525252005f;  // sqrt(5/(16pi))
constexpr float c2c = 0.54627421529603959f;  // sqrt(15/(16pi))
constexpr float c3a = 0.59004358992664352f;  // sqrt(35/(32pi))
constexpr float c3b = 2.8906114426405538f;   // sqrt(105/(4pi))
constexpr float c3c = 0.45704579946446572f;  // sqrt(21/(32pi))
constexpr float c3d = 0.37317633259011540f;  // sqrt(7/(16pi))
constexpr float c3e = 1.4453057213202769f;   // sqrt(105/(16pi))
}  // namespace shc

__device__ __forceinline__ void sh_basis(int deg, float x, float y, float z, float* Y)
{
    using namespace shc;
    Y[0] = c0;
    if (deg < 1) return;
    Y[1] = c1 * y;
    Y[2] = c1 * z;
    Y[3] = c1 * x;
    if (deg < 2) return;
    const float xx = x * x, yy = y * y, zz = z * z;
    Y[4] = c2a * x * y;
    Y[5] = c2a * y * z;
    Y[6] = c2b * (3.f * zz - 1.f);
    Y[7] = c2a * x * z;
    Y[8] = c2c * (xx - yy);
    if (deg < 3) return;
    Y[9] = c3a * y * (3.f * xx - yy);
    Y[10] = c3b * x * y * z;
    Y[11] = c3c * y * (5.f * zz - 1.f);
    Y[12] = c3d * z * (5.f * zz - 3.f);
    Y[13] = c3c * x * (5.f * zz - 1.f);
    Y[14] = c3e * z * (xx - yy);
    Y[15] = c3a * x * (xx - 3.f * yy);
}

// Gradient of each basis polynomial w.r.t. (x, y, z).
__device__ __forceinline__ void sh_basis_grad(int deg, float x, float y, float z, float (*dY)[3])
{
    using namespace shc;
    dY[0][0] = 0.f; dY[0][1] = 0.f; dY[0][2] = 0.f;
    if (deg < 1) return;
    dY[1][0] = 0.f; dY[1][1] = c1;  dY[1][2] = 0.f;
    dY[2][0] = 0.f; dY[2][1] = 0.f; dY[2][2] = c1;
    dY[3][0] = c1;  dY[3][1] = 0.f; dY[3][2] = 0.f;
    if (deg < 2) return;
    const float xx = x * x, yy = y * y, zz = z * z;
    dY[4][0] = c2a * y;       dY[4][1] = c2a * x;        dY[4][2] = 0.f;
    dY[5][0] = 0.f;           dY[5][1] = c2a * z;        dY[5][2] = c2a * y;
    dY[6][0] = 0.f;           dY[6][1] = 0.f;            dY[6][2] = 6.f * c2b * z;
    dY[7][0] = c2a * z;       dY[7][1] = 0.f;            dY[7][2] = c2a * x;
    dY[8][0] = 2.f * c2c * x; dY[8][1] = -2.f * c2c * y; dY[8][2] = 0.f;
    if (deg < 3) return;
    dY[9][0] = 6.f * c3a * x * y;  dY[9][1] = 3.f * c3a * (xx - yy);   dY[9][2] = 0.f;
    dY[10][0] = c3b * y * z;       dY[10][1] = c3b * x * z;            dY[10][2] = c3b * x * y;
    dY[11][0] = 0.f;               dY[11][1] = c3c * (5.f * zz - 1.f); dY[11][2] = 10.f * c3c * y * z;
    dY[12][0] = 0.f;               dY[12][1] = 0.f;                    dY[12][2] = c3d * (15.f * zz - 3.f);
    dY[13][0] = c3c * (5.f * zz - 1.f); dY[13][1] = 0.f;               dY[13][2] = 10.f * c3c * x * z;
    dY[14][0] = 2.f * c3e * x * z; dY[14][1] = -2.f * c3e * y * z;     dY[14][2] = c3e * (xx - yy);
    dY[15][0] = 3.f * c3a * (xx - yy); dY[15][1] = -6.f * c3a * x * y; dY[15][2] = 0.f;
}

// ---------------------------------------------------------------------------
// One fragment: the window value of a record at pixel offset (dx, dy).
// Forward and backward call exactly this code, so the alpha decisions of
// the backward replay those of the forward bit for bit.
// ---------------------------------------------------------------------------
struct Frag {
    float u;       // phi(p)/phi(s) (valid when > 0); the sigmoid: distance inside
    float lg;      // log2(u)
    float I;       // window
    float Ic;      // the sigmoid: 1 - I
    float oI;      // o * I before the clamp
    float a;       // alpha = min(alpha_max, o I)
    float w[3];    // LogSumExp: softmax weights of the three edges
    int k;         // edge that attains the minimum
};

__device__ __forceinline__ double edge_min(const double* A, const double* B, const double* C,
                                           double dx, double dy, int& k)
{
    const double u0 = fma(A[0], dx, fma(B[0], dy, C[0]));
    const double u1 = fma(A[1], dx, fma(B[1], dy, C[1]));
    const double u2 = fma(A[2], dx, fma(B[2], dy, C[2]));
    double u = u0;
    k = 0;
    if (u1 < u) { u = u1; k = 1; }
    if (u2 < u) { u = u2; k = 2; }
    return u;
}

__device__ __forceinline__ void window_alpha(float u, float o, float sigma, float alpha_max,
                                             Frag& f)
{
    f.u = u;
    f.lg = __builtin_amdgcn_logf(f.u);            // v_log_f32: log2
    f.I = __builtin_amdgcn_exp2f(sigma * f.lg);   // v_exp_f32: 2^x
    f.oI = o * f.I;
    f.a = fminf(alpha_max, f.oI);
}

// Sigmoid window (Eq. 2) at signed distance d inside the triangle (pixels):
// I = 1 / (1 + e), e = exp(-d / sigma), and 1 - I = e I.
__device__ __forceinline__ void sigmoid_alpha(double d64, float o, float sigma, float alpha_max,
                                              Frag& f)
{
    f.u = (float)d64;
    // 2^(-d log2(e) / sigma), the exponent capped at 64 so e stays finite
    // (I < 6e-20 beyond) and 1 - I = e I never becomes inf * 0
    const float e = __builtin_amdgcn_exp2f(
        fminf(f.u * __builtin_amdgcn_rcpf(sigma) * -1.4426950408889634f, 64.f));
    f.I = __builtin_amdgcn_rcpf(1.f + e);
    f.Ic = e * f.I;
    f.oI = o * f.I;
    f.a = fminf(alpha_max, f.oI);
}

// LogSumExp SDF in the window of Eq. 1: with d_k the distances inside,
// phi_lse = log sum_k exp(-d_k) = log sum_k exp(m - d_k) - m, m = min_k d_k
// (every exponent <= 0), u = phi_lse / phi_lse(s).  FP64 up to u: near the
// support's edge phi_lse is a small difference.  Returns u.
__device__ __forceinline__ double lse_u(const double* A, const double* B, const double* C,
                                        double dx, double dy, double phis, Frag& f)
{
    int k;
    const double m = edge_min(A, B, C, dx, dy, k);
    double e[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) e[j] = exp(m - fma(A[j], dx, fma(B[j], dy, C[j])));
    const double sum = (e[0] + e[1]) + e[2];
    const double inv = 1.0 / sum;
#pragma unroll
    for (int j = 0; j < 3; ++j) f.w[j] = (float)(e[j] * inv);
    f.k = k;
    return (log(sum) - m) / phis;
}

}  // namespace ts
