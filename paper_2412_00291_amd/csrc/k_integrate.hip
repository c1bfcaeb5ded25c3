// Per-map LiDAR integration kernels: block allocation (exact band-segment walk + hash),
// the projective TSDF update of Eq. 5 fused with block commit, dirty-set marking and the
// frame's bookkeeping, and camera label fusion (Eq. 6) for several cameras per launch.
// The bodies live in device.h and are shared with the batched kernels.
#include "device.h"

namespace mc {

// ---------------------------------------------------------------------------------
// pool initialisation and small helpers
// ---------------------------------------------------------------------------------

__global__ void k_fill_u64(unsigned long long *p, size_t n, unsigned long long v)
{
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = v;
}

hipError_t launch_fill_u64(unsigned long long *p, size_t n, unsigned long long v, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    size_t blocks = (n + kThreads - 1) / kThreads;
    int grid = (int)(blocks < 65536 ? blocks : 65536);
    hipLaunchKernelGGL(k_fill_u64, dim3(grid), dim3(kThreads), 0, s, p, n, v);
    return hipGetLastError();
}

// Fused labels start at 255 (unknown); D, W, counts and flags start at zero, which the
// caller clears with a device memset at create.
__global__ void k_init_fused(uint8_t *fused, size_t n)
{
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        reinterpret_cast<uint32_t *>(fused)[i] = 0xFFFFFFFFu;
}

hipError_t launch_init_pool(const MapView &m, hipStream_t s)
{
    size_t words = (size_t)m.max_blocks * kBlockVoxels / 4;
    size_t blocks = (words + kThreads - 1) / kThreads;
    int grid = (int)(blocks < 65536 ? blocks : 65536);
    hipLaunchKernelGGL(k_init_fused, dim3(grid), dim3(kThreads), 0, s, m.fused, words);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------------
// allocation: one thread per pixel, the workgroup's blocks de-duplicated in LDS
// ---------------------------------------------------------------------------------

__global__ __launch_bounds__(kThreads) void k_alloc(MapView m, FrameView f, LidarLUT L, Pose T,
                                                   const float *__restrict__ range)
{
    __shared__ unsigned long long lk[kLdsKeys];
    __shared__ int s_tmp[kThreads / 64];
    __shared__ unsigned long long s_base;
    for (int i = threadIdx.x; i < kLdsKeys; i += kThreads) lk[i] = kEmpty;
    __syncthreads();
    const int pix = blockIdx.x * kThreads + threadIdx.x;
    if (pix < L.rows * L.cols) alloc_pixel(lk, m, f, L, T, range, pix);
    __syncthreads();
    alloc_flush(lk, s_tmp, &s_base, m, f);
}

hipError_t launch_alloc(const MapView &m, const FrameView &f, const LidarLUT &lut, const Pose &T,
                        const float *range, hipStream_t s)
{
    int npix = lut.rows * lut.cols;
    int grid = (npix + kThreads - 1) / kThreads;
    hipLaunchKernelGGL(k_alloc, dim3(grid), dim3(kThreads), 0, s, m, f, lut, T, range);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------------
// TSDF integration: one workgroup per touched block (grid-stride); the last workgroup
// closes the frame
// ---------------------------------------------------------------------------------

__global__ __launch_bounds__(kThreads) void k_tsdf(MapView m, FrameView f, LidarLUT L, Pose T,
                                                  const float *__restrict__ range)
{
    __shared__ int s_slot;
    __shared__ int s_last;
    __shared__ unsigned long long s_sum[kThreads / 64];
    const FrameState fs = frame_state(m, f);
    unsigned long long my_updates = 0;
    for (int e = blockIdx.x; e < fs.n_list; e += gridDim.x) {
        const unsigned long long key = f.tk_key[e];
        if (threadIdx.x == 0) s_slot = commit_entry(m, f, fs, e, key);
        __syncthreads();
        if (fs.ok) {
            const int slot = s_slot;
            const int3 bc = unpack_key(key);
            if (threadIdx.x < 8) mark_neighbours(m, threadIdx.x, bc, slot, fs.epoch);
            float2 *dwb = m.dw + (size_t)slot * kBlockVoxels;
#pragma unroll
            for (int it = 0; it < kBlockVoxels / kThreads; ++it) {
                const int li = it * kThreads + threadIdx.x;
                bool band;
                my_updates += tsdf_voxel(m, L, T, range, dwb, bc, li, band);
                const unsigned long long bits = __ballot(band);
                if ((threadIdx.x & 63) == 0) f.band[(size_t)e * 8 + (li >> 6)] = bits;
            }
        }
        __syncthreads();
    }
    const unsigned long long w = wave_sum_u64(my_updates);
    if ((threadIdx.x & 63) == 0) s_sum[threadIdx.x >> 6] = w;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long t = 0;
        for (int i = 0; i < kThreads / 64; ++i) t += s_sum[i];
        if (t) atomicAdd(&m.ctr->updates, t);
        __threadfence();
        s_last = atomicAdd(&m.ctr->tsdf_done, 1u) == gridDim.x - 1;
    }
    __syncthreads();
    if (s_last && threadIdx.x == 0) {
        __threadfence();
        close_frame(m, fs);
        m.ctr->tsdf_done = 0;
    }
}

hipError_t launch_tsdf(const MapView &m, const FrameView &f, const LidarLUT &lut, const Pose &T,
                       const float *range, int grid, hipStream_t s)
{
    hipLaunchKernelGGL(k_tsdf, dim3(grid), dim3(kThreads), 0, s, m, f, lut, T, range);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------------
// label fusion: one workgroup per touched block, every camera of the call in order
// (equal to one call per camera: a voxel's votes are sequential)
// ---------------------------------------------------------------------------------

__global__ __launch_bounds__(kThreads) void k_labels(MapView m, FrameView f, CameraSet cs)
{
    __shared__ unsigned long long s_sum[kThreads / 64];
    const int n = m.ctr->last_touched;
    unsigned long long my_votes = 0;
    for (int e = blockIdx.x; e < n; e += gridDim.x) {
        const int slot = f.tk_slot[e];
        const int3 bc = unpack_key(f.tk_key[e]);
#pragma unroll
        for (int it = 0; it < kBlockVoxels / kThreads; ++it) {
            const int li = it * kThreads + threadIdx.x;
            const unsigned long long bits = f.band[(size_t)e * 8 + (li >> 6)];
            if (bits == 0) continue;  // wave-uniform: one word per wave
            if ((bits >> (li & 63)) & 1ull) my_votes += label_voxel(m, cs, slot, bc, li);
        }
    }
    unsigned long long w = wave_sum_u64(my_votes);
    if ((threadIdx.x & 63) == 0) s_sum[threadIdx.x >> 6] = w;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long t = 0;
        for (int i = 0; i < kThreads / 64; ++i) t += s_sum[i];
        if (t) atomicAdd(&m.ctr->votes, t);
    }
}

hipError_t launch_labels(const MapView &m, const FrameView &f, const CameraSet &cams, int grid, hipStream_t s)
{
    hipLaunchKernelGGL(k_labels, dim3(grid), dim3(kThreads), 0, s, m, f, cams);
    return hipGetLastError();
}

}  // namespace mc
