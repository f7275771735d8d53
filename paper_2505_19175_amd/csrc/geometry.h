// geometry.h -- per-triangle geometry shared by the projection and the
// backward projection (internal): camera-space and projected vertices, edge
// vectors and lengths, the depth key, the view direction, SH row loads.
#pragma once

#include "ts_device.h"

namespace ts {

// Camera-space and projected vertices with the edge quantities every
// consumer needs.  Edge k runs from q_k to q_{k+1}.
struct Geo {
    double xc[3][3];
    double q[3][2];
    double e[3][2];
    double len[3];
    double S;     // signed doubled area
    double P;     // perimeter
    bool front;   // every vertex beyond the near plane
};

__device__ __forceinline__ void load_vertices(const float* __restrict__ v, int64_t i, float vv[9])
{
    const float* p = v + 9 * i;
#pragma unroll
    for (int a = 0; a < 9; ++a) vv[a] = p[a];
}

__device__ __forceinline__ void project_geo(const float vv[9], const Cam& cam, float z_near, Geo& g)
{
    g.front = true;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            double acc = (double)cam.t[a];
            acc = fma((double)cam.R[3 * a + 0], (double)vv[3 * j + 0], acc);
            acc = fma((double)cam.R[3 * a + 1], (double)vv[3 * j + 1], acc);
            acc = fma((double)cam.R[3 * a + 2], (double)vv[3 * j + 2], acc);
            g.xc[j][a] = acc;
        }
        g.front = g.front && (g.xc[j][2] > (double)z_near);
        const double iz = 1.0 / g.xc[j][2];
        g.q[j][0] = fma((double)cam.fx * g.xc[j][0], iz, (double)cam.cx);
        g.q[j][1] = fma((double)cam.fy * g.xc[j][1], iz, (double)cam.cy);
    }
    g.P = 0.0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const int k1 = k == 2 ? 0 : k + 1;
        g.e[k][0] = g.q[k1][0] - g.q[k][0];
        g.e[k][1] = g.q[k1][1] - g.q[k][1];
        g.len[k] = sqrt(g.e[k][0] * g.e[k][0] + g.e[k][1] * g.e[k][1]);
        g.P += g.len[k];
    }
    // 2A = cross(q1 - q0, q2 - q0)
    g.S = g.e[0][0] * (g.q[2][1] - g.q[0][1]) - g.e[0][1] * (g.q[2][0] - g.q[0][0]);
}

// Depth key: mean camera-space z of the three vertices, every operation
// rounded in the written order (no contraction), so the float32 key is a
// fixed function of the inputs: z_j = ((R20 v0 + R21 v1) + R22 v2) + t2,
// z_c = ((z_0 + z_1) + z_2) / 3.
__device__ __forceinline__ double depth_centre(const float vv[9], const Cam& cam)
{
    double zs = 0.0;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        double z = __dmul_rn((double)cam.R[6], (double)vv[3 * j + 0]);
        z = __dadd_rn(z, __dmul_rn((double)cam.R[7], (double)vv[3 * j + 1]));
        z = __dadd_rn(z, __dmul_rn((double)cam.R[8], (double)vv[3 * j + 2]));
        z = __dadd_rn(z, (double)cam.t[2]);
        zs = j == 0 ? z : __dadd_rn(zs, z);
    }
    return zs / 3.0;
}

// Unit direction from the camera centre -R^T t to the centroid, and its norm.
__device__ __forceinline__ void view_dir(const float vv[9], const Cam& cam, double d[3], double& nrm)
{
    double dv[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double cen = ((double)vv[a] + (double)vv[3 + a] + (double)vv[6 + a]) * (1.0 / 3.0);
        const double cc = -((double)cam.R[a] * cam.t[0] + (double)cam.R[3 + a] * cam.t[1] +
                            (double)cam.R[6 + a] * cam.t[2]);
        dv[a] = cen - cc;
    }
    nrm = sqrt(dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2]);
#pragma unroll
    for (int a = 0; a < 3; ++a) d[a] = dv[a] / nrm;
}

// Coefficients of one triangle: float4 loads when the row is 16-byte aligned.
template <int DEG>
__device__ __forceinline__ void load_sh(const float* __restrict__ sh, int64_t i, float* c)
{
    constexpr int NSH = 3 * (DEG + 1) * (DEG + 1);
    const float* p = sh + (int64_t)NSH * i;
    if constexpr (NSH % 4 == 0) {
        const float4* q = reinterpret_cast<const float4*>(p);
#pragma unroll
        for (int j = 0; j < NSH / 4; ++j) {
            const float4 t = q[j];
            c[4 * j + 0] = t.x; c[4 * j + 1] = t.y; c[4 * j + 2] = t.z; c[4 * j + 3] = t.w;
        }
    } else {
#pragma unroll
        for (int j = 0; j < NSH; ++j) c[j] = p[j];
    }
}

}  // namespace ts
