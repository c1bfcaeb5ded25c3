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
// TSDF integration over the touched blocks (grid-stride); the last workgroup closes the
// frame.  kSched 0: one workgroup per block (two voxels per thread); 1: one wavefront per
// block (eight voxels per lane, four blocks in flight per workgroup).
// ---------------------------------------------------------------------------------

template <int kSched>
__global__ __launch_bounds__(kThreads) void k_tsdf(MapView m, FrameView f, LidarLUT L, Pose T,
                                                  const float *__restrict__ range, uint32_t frame_id)
{
    __shared__ int s_slot;
    __shared__ int s_last;
    __shared__ unsigned long long s_sum[kThreads / 64];
    const FrameState fs = frame_state(m, f);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    constexpr int kWidth = kSched == 0 ? kThreads : 64;
    const int rank = kSched == 0 ? (int)threadIdx.x : lane;
    const int first = kSched == 0 ? (int)blockIdx.x : (int)blockIdx.x * (kThreads / 64) + wave;
    const int stride = kSched == 0 ? (int)gridDim.x : (int)gridDim.x * (kThreads / 64);
    unsigned long long my_updates = 0;
    for (int e = first; e < fs.n_list; e += stride) {
        const unsigned long long key = f.tk_key[e];
        int slot;
        if (kSched == 0) {
            if (threadIdx.x == 0) s_slot = commit_entry(m, f, fs, e, key, frame_id);
            __syncthreads();
            slot = s_slot;
        } else {
            slot = 0;
            if (lane == 0) slot = commit_entry(m, f, fs, e, key, frame_id);
            slot = __shfl(slot, 0, 64);
        }
        if (fs.ok) {
            const int3 bc = unpack_key(key);
            if (rank < 8) mark_neighbours(m, rank, bc, slot, fs.epoch, frame_id);
            float2 *dwb = m.dw + (size_t)slot * kBlockVoxels;
#pragma unroll
            for (int it = 0; it < kBlockVoxels / kWidth; ++it) {
                const int li = it * kWidth + rank;
                bool band;
                my_updates += tsdf_voxel(m, L, T, range, dwb, bc, li, band);
                const unsigned long long bits = __ballot(band);
                if (lane == 0) f.band[(size_t)e * 8 + (li >> 6)] = bits;
            }
        }
        if (kSched == 0) __syncthreads();
    }
    const unsigned long long w = wave_sum_u64(my_updates);
    if (lane == 0) s_sum[wave] = w;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long t = 0;
        for (int i = 0; i < kThreads / 64; ++i) t += s_sum[i];
        if (t) atomicAdd(&m.ctr->updates, t);
        wait_memory();  // the update count lands before the ticket
        s_last = atomicAdd(&m.ctr->tsdf_done, 1u) == gridDim.x - 1;
    }
    __syncthreads();
    if (s_last && threadIdx.x == 0) {
        close_frame(m, fs);
        m.ctr->tsdf_done = 0;
    }
}

hipError_t launch_tsdf(const MapView &m, const FrameView &f, const LidarLUT &lut, const Pose &T,
                       const float *range, uint32_t frame_id, int schedule, int grid, hipStream_t s)
{
    if (schedule == 0) hipLaunchKernelGGL(k_tsdf<0>, dim3(grid), dim3(kThreads), 0, s, m, f, lut, T, range, frame_id);
    else hipLaunchKernelGGL(k_tsdf<1>, dim3(grid), dim3(kThreads), 0, s, m, f, lut, T, range, frame_id);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------------
// label fusion over the last frame's touched blocks, every camera of the call in order
// (equal to one call per camera: a voxel's votes are sequential); schedules as above
// ---------------------------------------------------------------------------------

template <int kSched>
__global__ __launch_bounds__(kThreads) void k_labels(MapView m, FrameView f, CameraSet cs)
{
    __shared__ unsigned long long s_sum[kThreads / 64];
    const int n = m.ctr->last_touched;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    constexpr int kWidth = kSched == 0 ? kThreads : 64;
    const int rank = kSched == 0 ? (int)threadIdx.x : lane;
    const int first = kSched == 0 ? (int)blockIdx.x : (int)blockIdx.x * (kThreads / 64) + wave;
    const int stride = kSched == 0 ? (int)gridDim.x : (int)gridDim.x * (kThreads / 64);
    unsigned long long my_votes = 0;
    for (int e = first; e < n; e += stride) {
        const int slot = f.tk_slot[e];
        const int3 bc = unpack_key(f.tk_key[e]);
#pragma unroll
        for (int it = 0; it < kBlockVoxels / kWidth; ++it) {
            const int li = it * kWidth + rank;
            const unsigned long long bits = f.band[(size_t)e * 8 + (li >> 6)];
            if (bits == 0) continue;  // wave-uniform: one word per wave
            if ((bits >> (li & 63)) & 1ull) my_votes += label_voxel(m, cs, slot, bc, li);
        }
    }
    unsigned long long w = wave_sum_u64(my_votes);
    if (lane == 0) s_sum[wave] = w;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long t = 0;
        for (int i = 0; i < kThreads / 64; ++i) t += s_sum[i];
        if (t) atomicAdd(&m.ctr->votes, t);
    }
}

hipError_t launch_labels(const MapView &m, const FrameView &f, const CameraSet &cams, int schedule, int grid,
                         hipStream_t s)
{
    if (schedule == 0) hipLaunchKernelGGL(k_labels<0>, dim3(grid), dim3(kThreads), 0, s, m, f, cams);
    else hipLaunchKernelGGL(k_labels<1>, dim3(grid), dim3(kThreads), 0, s, m, f, cams);
    return hipGetLastError();
}

}  // namespace mc
