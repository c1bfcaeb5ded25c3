// Trilinear SDF query and its SE(3) pose / point adjoint.
//
// The distance field is sampled at voxel centres x = nu v (Sec. IV-C.2); a point x is
// interpolated trilinearly from the eight voxels around q = x / nu (lerp along x, then
// y, then z) and is valid only when all eight are observed (W > 0).  For a posed scan
// y_j = Exp(w) p_j + t the loss is sum_j D(y_j)^2; its gradient is
//   g_j = 2 D grad D,  dL/dt = sum g_j,  dL/dw = J_l(w)^T sum (R p_j) x g_j,
//   dL/dp_j = R^T g_j,
// with J_l the left Jacobian of SO(3).  Per-pose sums are reduced in a fixed order.
#include "device.h"

namespace mc {

// trilinear sample at voxel-space point q; grad is dD/dx (already divided by nu)
__device__ __forceinline__ bool sample(const MapView &m, float qx, float qy, float qz, float &D, float g[3])
{
    const float lim = (float)kDomainVoxels;
    if (!(fabsf(qx) < lim && fabsf(qy) < lim && fabsf(qz) < lim)) return false;
    const float fx0 = floorf(qx), fy0 = floorf(qy), fz0 = floorf(qz);
    const float fx = qx - fx0, fy = qy - fy0, fz = qz - fz0;
    const int x0 = (int)fx0, y0 = (int)fy0, z0 = (int)fz0;
    float Dc[8];
    unsigned long long last_key = kEmpty;
    int last_slot = -1;
#pragma unroll
    for (int n = 0; n < 8; ++n) {
        const int vx = x0 + (n & 1), vy = y0 + ((n >> 1) & 1), vz = z0 + ((n >> 2) & 1);
        const unsigned long long key = pack_key(vx >> 3, vy >> 3, vz >> 3);
        if (key != last_key) {
            last_key = key;
            last_slot = hash_find(m, key);
        }
        if (last_slot < 0) return false;
        const float2 v = m.dw[(size_t)last_slot * kBlockVoxels + (vx & 7) + 8 * (vy & 7) + 64 * (vz & 7)];
        if (!(v.y > 0.0f)) return false;
        Dc[n] = v.x;
    }
    const float c00 = Dc[0] + fx * (Dc[1] - Dc[0]), c10 = Dc[2] + fx * (Dc[3] - Dc[2]);
    const float c01 = Dc[4] + fx * (Dc[5] - Dc[4]), c11 = Dc[6] + fx * (Dc[7] - Dc[6]);
    const float c0 = c00 + fy * (c10 - c00), c1 = c01 + fy * (c11 - c01);
    D = c0 + fz * (c1 - c0);
    const float gx00 = Dc[1] - Dc[0], gx10 = Dc[3] - Dc[2], gx01 = Dc[5] - Dc[4], gx11 = Dc[7] - Dc[6];
    const float gx0 = gx00 + fy * (gx10 - gx00), gx1 = gx01 + fy * (gx11 - gx01);
    g[0] = (gx0 + fz * (gx1 - gx0)) / m.nu;
    g[1] = ((c10 - c00) + fz * ((c11 - c01) - (c10 - c00))) / m.nu;
    g[2] = (c1 - c0) / m.nu;
    return true;
}

__global__ __launch_bounds__(kThreads) void k_query(MapView m, const float *__restrict__ pts, long long n,
                                                   float *sdf, float *grad, uint8_t *valid)
{
    for (long long i = blockIdx.x * (long long)kThreads + threadIdx.x; i < n; i += (long long)gridDim.x * kThreads) {
        const float x = pts[3 * i], y = pts[3 * i + 1], z = pts[3 * i + 2];
        float D = 0.0f, g[3] = {0.0f, 0.0f, 0.0f};
        const bool ok = sample(m, x / m.nu, y / m.nu, z / m.nu, D, g);
        if (!ok) { D = 0.0f; g[0] = g[1] = g[2] = 0.0f; }
        sdf[i] = D;
        if (grad) {
            grad[3 * i] = g[0];
            grad[3 * i + 1] = g[1];
            grad[3 * i + 2] = g[2];
        }
        valid[i] = ok ? 1 : 0;
    }
}

hipError_t launch_query(const MapView &m, const float *pts, long long n, float *sdf, float *grad,
                        uint8_t *valid, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    long long blocks = (n + kThreads - 1) / kThreads;
    int grid = (int)(blocks < 8192 ? blocks : 8192);
    hipLaunchKernelGGL(k_query, dim3(grid), dim3(kThreads), 0, s, m, pts, n, sdf, grad, valid);
    return hipGetLastError();
}

// Exp(w) and the left Jacobian J_l(w) in fp32: the series is used up to |w| = 0.5 (its
// truncation error there is ~1e-13), the closed forms above it.
__device__ void so3_exp_jl(const float w[3], float R[9], float J[9])
{
    const float th2 = w[0] * w[0] + w[1] * w[1] + w[2] * w[2];
    const float th = sqrtf(th2);
    float A, B, C;  // sin t / t, (1 - cos t) / t^2, (t - sin t) / t^3
    if (th < 0.5f) {
        const float t4 = th2 * th2, t6 = t4 * th2, t8 = t4 * t4;
        A = 1.0f - th2 / 6.0f + t4 / 120.0f - t6 / 5040.0f + t8 / 362880.0f;
        B = 0.5f - th2 / 24.0f + t4 / 720.0f - t6 / 40320.0f + t8 / 3628800.0f;
        C = 1.0f / 6.0f - th2 / 120.0f + t4 / 5040.0f - t6 / 362880.0f + t8 / 39916800.0f;
    } else {
        const float sh = sinf(0.5f * th), s = sinf(th);
        A = s / th;
        B = 2.0f * sh * sh / th2;
        C = (th - s) / (th2 * th);
    }
    const float K[9] = {0.0f, -w[2], w[1], w[2], 0.0f, -w[0], -w[1], w[0], 0.0f};
    float K2[9];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
            K2[3 * i + j] = (K[3 * i] * K[j] + K[3 * i + 1] * K[3 + j]) + K[3 * i + 2] * K[6 + j];
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const float I = (i % 4 == 0) ? 1.0f : 0.0f;
        R[i] = (I + A * K[i]) + B * K2[i];
        J[i] = (I + B * K[i]) + C * K2[i];
    }
}

// partial sums per (pose, chunk): loss, dL/dt (3), sum (R p) x g (3), pad
__global__ __launch_bounds__(kThreads) void k_adjoint(MapView m, const float *__restrict__ xi,
                                                     const float *__restrict__ pts, long long N, float *gpts,
                                                     float *partial)
{
    __shared__ float sR[9];
    __shared__ float red[8][kThreads];
    const int b = blockIdx.y;
    if (threadIdx.x == 0) {
        float w[3] = {xi[6 * b + 3], xi[6 * b + 4], xi[6 * b + 5]}, J[9];
        so3_exp_jl(w, sR, J);
    }
    __syncthreads();
    const float t0 = xi[6 * b], t1 = xi[6 * b + 1], t2 = xi[6 * b + 2];
    float acc[7] = {0, 0, 0, 0, 0, 0, 0};
    const long long j = blockIdx.x * (long long)kThreads + threadIdx.x;
    if (j < N) {
        const float *p = pts + ((size_t)b * N + j) * 3;
        const float px = p[0], py = p[1], pz = p[2];
        float Rp[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) Rp[i] = (sR[3 * i] * px + sR[3 * i + 1] * py) + sR[3 * i + 2] * pz;
        const float y0 = Rp[0] + t0, y1 = Rp[1] + t1, y2 = Rp[2] + t2;
        float D, g[3];
        float gp[3] = {0.0f, 0.0f, 0.0f};
        if (sample(m, y0 / m.nu, y1 / m.nu, y2 / m.nu, D, g)) {
            const float gg[3] = {2.0f * D * g[0], 2.0f * D * g[1], 2.0f * D * g[2]};
            acc[0] = D * D;
            acc[1] = gg[0];
            acc[2] = gg[1];
            acc[3] = gg[2];
            acc[4] = Rp[1] * gg[2] - Rp[2] * gg[1];
            acc[5] = Rp[2] * gg[0] - Rp[0] * gg[2];
            acc[6] = Rp[0] * gg[1] - Rp[1] * gg[0];
#pragma unroll
            for (int i = 0; i < 3; ++i) gp[i] = (sR[i] * gg[0] + sR[3 + i] * gg[1]) + sR[6 + i] * gg[2];
        }
        if (gpts) {
            float *o = gpts + ((size_t)b * N + j) * 3;
            o[0] = gp[0];
            o[1] = gp[1];
            o[2] = gp[2];
        }
    }
#pragma unroll
    for (int k = 0; k < 7; ++k) red[k][threadIdx.x] = acc[k];
    __syncthreads();
    for (int s = kThreads / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s)
#pragma unroll
            for (int k = 0; k < 7; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x < 8) partial[((size_t)b * gridDim.x + blockIdx.x) * 8 + threadIdx.x] =
        threadIdx.x < 7 ? red[threadIdx.x][0] : 0.0f;
}

hipError_t launch_adjoint(const MapView &m, const float *xi, const float *pts, int B, long long N,
                          float *gpts, float *partial, int nchunk, hipStream_t s)
{
    hipLaunchKernelGGL(k_adjoint, dim3(nchunk, B), dim3(kThreads), 0, s, m, xi, pts, N, gpts, partial);
    return hipGetLastError();
}

__global__ __launch_bounds__(kThreads) void k_adjoint_reduce(const float *__restrict__ xi,
                                                            const float *__restrict__ partial, int nchunk,
                                                            float *loss, float *gxi)
{
    __shared__ float red[7][kThreads];
    const int b = blockIdx.x;
    float acc[7] = {0, 0, 0, 0, 0, 0, 0};
    for (int c = threadIdx.x; c < nchunk; c += kThreads)
#pragma unroll
        for (int k = 0; k < 7; ++k) acc[k] += partial[((size_t)b * nchunk + c) * 8 + k];
#pragma unroll
    for (int k = 0; k < 7; ++k) red[k][threadIdx.x] = acc[k];
    __syncthreads();
    for (int s = kThreads / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s)
#pragma unroll
            for (int k = 0; k < 7; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        float w[3] = {xi[6 * b + 3], xi[6 * b + 4], xi[6 * b + 5]}, R[9], J[9];
        so3_exp_jl(w, R, J);
        loss[b] = red[0][0];
        gxi[6 * b] = red[1][0];
        gxi[6 * b + 1] = red[2][0];
        gxi[6 * b + 2] = red[3][0];
        const float m0 = red[4][0], m1 = red[5][0], m2 = red[6][0];
        for (int i = 0; i < 3; ++i) gxi[6 * b + 3 + i] = (J[i] * m0 + J[3 + i] * m1) + J[6 + i] * m2;
    }
}

hipError_t launch_adjoint_reduce(const float *xi, const float *partial, int B, int nchunk, float *loss,
                                 float *gxi, hipStream_t s)
{
    hipLaunchKernelGGL(k_adjoint_reduce, dim3(B), dim3(kThreads), 0, s, xi, partial, nchunk, loss, gxi);
    return hipGetLastError();
}

}  // namespace mc
