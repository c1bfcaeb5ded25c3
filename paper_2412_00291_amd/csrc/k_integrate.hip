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

// kNP: the non-projective distance, whose normal image and point filter are computed here
// (one pixel per thread, stored in the frame's normal image for the TSDF pass).
template <bool kNP>
__global__ __launch_bounds__(kThreads) void k_alloc(MapView m, FrameView f, LidarLUT L, Pose T,
                                                   const float *__restrict__ range, float cos_inc)
{
    __shared__ unsigned long long lk[kLdsKeys];
    __shared__ int s_tmp[kThreads / 64];
    __shared__ unsigned long long s_base;
    // the frame starts: the previous frame's label votes are cleared here (its label launches
    // have completed), so the TSDF launch, which may fuse this frame's labels, keeps its own
    if (blockIdx.x == 0 && threadIdx.x < 64) (void)spread_take_wave(m.sync->votes);
    for (int i = threadIdx.x; i < kLdsKeys; i += kThreads) lk[i] = kEmpty;
    __syncthreads();
    const int pix = blockIdx.x * kThreads + threadIdx.x;
    if (pix < L.rows * L.cols) alloc_pixel<kNP, true>(lk, m, f, L, T, range, pix, cos_inc);
    __syncthreads();
    alloc_flush(lk, s_tmp, &s_base, m, f);
}

hipError_t launch_alloc(const MapView &m, const FrameView &f, const LidarLUT &lut, const Pose &T,
                        const float *range, int dist_mode, float cos_inc, hipStream_t s)
{
    int npix = lut.rows * lut.cols;
    int grid = (npix + kThreads - 1) / kThreads;
    if (dist_mode == kDistNonProjective)
        hipLaunchKernelGGL(k_alloc<true>, dim3(grid), dim3(kThreads), 0, s, m, f, lut, T, range, cos_inc);
    else
        hipLaunchKernelGGL(k_alloc<false>, dim3(grid), dim3(kThreads), 0, s, m, f, lut, T, range, cos_inc);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------------
// TSDF integration over the touched blocks (grid-stride); the last workgroup (by a
// hierarchical ticket) closes the frame.  A worker is a workgroup (kSched 0, two voxels per thread) or a wavefront
// (kSched 1, eight voxels per lane, four workers per workgroup).  A worker takes its
// entries a chunk at a time: the chunk's commits run on one lane each, then the voxels of
// each entry in turn, then the neighbour marks on eight lanes per entry, all at once.
// ---------------------------------------------------------------------------------

// The nearest-pixel search reads the column and row boundary tables for every voxel; a
// workgroup copies them (cols + rows + 1 pairs, 17 KiB for 2048 columns) into dynamic LDS
// when the launch provides it (kLdsLut), so that the range image is the voxel's only
// global read on the way to its update.
// kLab: label fusion of the frame's camera label images fused into the pass (0 none, 1 vote
// counts, 2 latest label): the band words of a chunk's blocks are gathered in LDS while
// the blocks are updated, and after the chunk's updates the worker takes all of their band
// voxels as one flat list and votes them exactly as the label kernel would (the votes of
// a voxel depend only on that voxel), so a chunk's label reads are one latency chain.
template <int kN>
struct ChunkBand {
    unsigned long long w[kN][8];  // band words of the chunk's blocks
    int pre[kN][9];               // prefix of each block's word popcounts
    int epre[kN + 1];             // prefix of the blocks' band voxels
    int slot[kN];
    int3 bc[kN];
};

// Band voxel t (< the chunk's total) of the chunk: block j, voxel li.
template <int kN>
__device__ __forceinline__ void chunk_band_voxel(const ChunkBand<kN> &g, int n, int t, int &j, int &li)
{
    int lo = 0, hi = n - 1;  // last block whose prefix is <= t
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (g.epre[mid] <= t) lo = mid;
        else hi = mid - 1;
    }
    j = lo;
    const int local = t - g.epre[j];
    int k = 0;
#pragma unroll
    for (int i = 1; i < 8; ++i) k += g.pre[j][i] <= local ? 1 : 0;
    li = band_bit(g.w[j][k], k, local - g.pre[j][k]);
}
template <int kSched, bool kLdsLut, bool kNP, int kLab>
__global__ __launch_bounds__(kThreads) void k_tsdf(MapView m, FrameView f, LidarLUT L, Pose T,
                                                  const float *__restrict__ range, uint32_t frame_id, CameraSet cs)
{
    constexpr int kWidth = kSched == 0 ? kThreads : 64;
    constexpr int kChunk = kWidth / 8;  // entries per chunk: eight marking lanes each
    extern __shared__ float2 s_lut[];
    __shared__ int s_slot[kThreads / 8];
    __shared__ unsigned long long s_sum[kThreads / 64];
    __shared__ unsigned long long s_vsum[kThreads / 64];
    __shared__ ChunkBand<kLab ? kChunk : 1> s_cb[kLab ? (kSched == 0 ? 1 : kThreads / 64) : 1];
    const FrameRaw raw = frame_raw(m);  // in flight with the table copy
    if (kLdsLut) stage_lut(L, s_lut);
    const FrameState fs = frame_state_of(raw, m, f);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int rank = kSched == 0 ? (int)threadIdx.x : lane;
    const int first = kSched == 0 ? (int)blockIdx.x : (int)blockIdx.x * (kThreads / 64) + wave;
    const int stride = kSched == 0 ? (int)gridDim.x : (int)gridDim.x * (kThreads / 64);
    unsigned long long my_updates = 0, my_votes = 0;
    auto &cb = s_cb[kLab && kSched != 0 ? wave : 0];
    for (int base = first; base < fs.n_list; base += kChunk * stride) {
        int my_slot = -1;  // lane i < kChunk commits entry base + i * stride
        const int ec = base + rank * stride;
        if (rank < kChunk && ec < fs.n_list) my_slot = commit_entry(m, f, fs, ec, f.tk_key[ec], frame_id);
        if (kSched == 0) {
            if (rank < kChunk) s_slot[rank] = my_slot;
            __syncthreads();
        }
        if (fs.ok) {
            for (int j = 0; j < kChunk; ++j) {
                const int e = base + j * stride;
                if (e >= fs.n_list) break;
                const int slot = kSched == 0 ? s_slot[j] : __shfl(my_slot, j, 64);
                const unsigned long long key = f.tk_key[e];
                my_updates += tsdf_block<kWidth, kNP>(m, f, L, T, range, e, key, slot, rank,
                                                       kLab ? cb.w[j] : nullptr);
                if (kLab && rank == 0) {
                    cb.slot[j] = slot;
                    cb.bc[j] = unpack_key(key);
                }
            }
            if (kLab) {  // the chunk's band voxels as one flat list
                const int nE = min(kChunk, (fs.n_list - base + stride - 1) / stride);
                if (kSched == 0) __syncthreads();
                else __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                if (rank < nE) {
                    int p = 0;
                    cb.pre[rank][0] = 0;
#pragma unroll
                    for (int k = 0; k < 8; ++k) {
                        p += __popcll(cb.w[rank][k]);
                        cb.pre[rank][k + 1] = p;
                    }
                }
                if (kSched == 0) __syncthreads();
                else __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                if (rank == 0) {
                    int p = 0;
                    for (int j = 0; j < nE; ++j) {
                        cb.epre[j] = p;
                        p += cb.pre[j][8];
                    }
                    cb.epre[nE] = p;
                }
                if (kSched == 0) __syncthreads();
                else __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
#pragma unroll 1
                for (int t = rank; t < cb.epre[nE]; t += kWidth) {
                    int j, li;
                    chunk_band_voxel(cb, nE, t, j, li);
                    my_votes += kLab == 2 ? label_voxel_latest(m, cs, cb.slot[j], cb.bc[j], li)
                                          : label_voxel(m, cs, cb.slot[j], cb.bc[j], li);
                }
            }
            // dirty marks last: nothing above waits for their hash probes
            const int i = rank >> 3;  // lane r marks neighbour r % 8 of entry r / 8
            const int em = base + i * stride;
            const int si = kSched == 0 ? s_slot[i] : __shfl(my_slot, i, 64);
            if (em < fs.n_list) {
                const int s = neighbour_slot(m, rank & 7, unpack_key(f.tk_key[em]), si, frame_id);
                if (s >= 0) mark_dirty(m, s, fs.epoch, fs.bits);
            }
        }
        if (kSched == 0) __syncthreads();  // s_slot is rewritten by the next chunk
    }
    const unsigned long long w = wave_sum_u64(my_updates);
    const unsigned long long wv = kLab ? wave_sum_u64(my_votes) : 0ull;
    if (lane == 0) {
        s_sum[wave] = w;
        s_vsum[wave] = wv;
    }
    __syncthreads();
    if (threadIdx.x == 0) {  // the last workgroup closes the frame with the launch's update count
        unsigned long long t = 0, tv = 0;
        for (int i = 0; i < kThreads / 64; ++i) {
            t += s_sum[i];
            tv += s_vsum[i];
        }
        if (kLab && tv) spread_add(m.sync->votes, tv);
        unsigned long long total = 0;
        if (ticket_arrive_sum(m.sync->tsdf, t, &total)) close_frame(m, fs, total);
    }
}

template <bool kNP, int kLab>
static void launch_tsdf_t(const MapView &m, const FrameView &f, const LidarLUT &lut, const Pose &T,
                          const float *range, uint32_t frame_id, int schedule, int grid, const CameraSet &cs,
                          hipStream_t s)
{
    const size_t lds = ((size_t)lut.cols + lut.rows + 1) * sizeof(float2);
    if (lds <= kMaxLdsLut) {
        if (schedule == 0)
            hipLaunchKernelGGL((k_tsdf<0, true, kNP, kLab>), dim3(grid), dim3(kThreads), lds, s, m, f, lut, T, range,
                               frame_id, cs);
        else
            hipLaunchKernelGGL((k_tsdf<1, true, kNP, kLab>), dim3(grid), dim3(kThreads), lds, s, m, f, lut, T, range,
                               frame_id, cs);
    } else {
        if (schedule == 0)
            hipLaunchKernelGGL((k_tsdf<0, false, kNP, kLab>), dim3(grid), dim3(kThreads), 0, s, m, f, lut, T, range,
                               frame_id, cs);
        else
            hipLaunchKernelGGL((k_tsdf<1, false, kNP, kLab>), dim3(grid), dim3(kThreads), 0, s, m, f, lut, T, range,
                               frame_id, cs);
    }
}

template <bool kNP>
static void launch_tsdf_l(const MapView &m, const FrameView &f, const LidarLUT &lut, const Pose &T,
                          const float *range, uint32_t frame_id, int schedule, int grid, const CameraSet &cs,
                          int label_mode, hipStream_t s)
{
    if (cs.n == 0) launch_tsdf_t<kNP, 0>(m, f, lut, T, range, frame_id, schedule, grid, cs, s);
    else if (label_mode == kLabelLatest) launch_tsdf_t<kNP, 2>(m, f, lut, T, range, frame_id, schedule, grid, cs, s);
    else launch_tsdf_t<kNP, 1>(m, f, lut, T, range, frame_id, schedule, grid, cs, s);
}

hipError_t launch_tsdf(const MapView &m, const FrameView &f, const LidarLUT &lut, const Pose &T,
                       const float *range, uint32_t frame_id, int schedule, int grid, int dist_mode,
                       const CameraSet &cams, int label_mode, hipStream_t s)
{
    if (dist_mode == kDistNonProjective)
        launch_tsdf_l<true>(m, f, lut, T, range, frame_id, schedule, grid, cams, label_mode, s);
    else
        launch_tsdf_l<false>(m, f, lut, T, range, frame_id, schedule, grid, cams, label_mode, s);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------------
// label fusion over the last frame's touched blocks, every camera of the call in order
// (equal to one call per camera: a voxel's votes are sequential); a worker takes a block's
// band voxels compacted (about one in ten voxels is in the band); schedules as above
// ---------------------------------------------------------------------------------

// The band voxels of the last frame's touched entries, each passed to vote(slot, bc, li)
// (which returns its votes); the votes go to the map's spread counter.  kSched 0: a
// workgroup takes its entries blockIdx + j G kLabGroup at a time with their voxels as one
// flat list; kSched 1: a wavefront takes one entry at a time.
template <int kSched, class Vote>
__device__ __forceinline__ void for_band_voxels(const MapView &m, const FrameView &f, Vote vote)
{
    __shared__ unsigned long long s_sum[kThreads / 64];
    __shared__ LabelGroup g;
    const int n = m.ctr->last_touched;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    unsigned long long my_votes = 0;
    if (kSched == 0) {
        const int G = (int)gridDim.x;
        for (int e0 = blockIdx.x; e0 < n; e0 += kLabGroup * G) {
            {  // all of the group's reads at once (clamped indices, masked after)
                const int j = (threadIdx.x >> 3) & (kLabGroup - 1), k = threadIdx.x & 7;
                const int ew = e0 + j * G, es = e0 + (int)(threadIdx.x & (kLabGroup - 1)) * G;
                const bool okw = threadIdx.x < kLabGroup * 8 && ew < n, oks = es < n;
                const unsigned long long wv = f.band[okw ? (size_t)ew * 8 + k : 0];
                const int sv = f.tk_slot[oks ? es : 0];
                const unsigned long long kv = f.tk_key[oks ? es : 0];
                if (threadIdx.x < kLabGroup * 8) g.w[j][k] = okw ? wv : 0ull;
                if (threadIdx.x < kLabGroup) {
                    g.slot[threadIdx.x] = oks ? sv : -1;
                    g.key[threadIdx.x] = oks ? kv : 0ull;
                }
            }
            __syncthreads();
            if (threadIdx.x < kLabGroup) {
                int p = 0;
                g.pre[threadIdx.x][0] = 0;
#pragma unroll
                for (int k = 0; k < 8; ++k) {
                    p += __popcll(g.w[threadIdx.x][k]);
                    g.pre[threadIdx.x][k + 1] = p;
                }
            }
            __syncthreads();
            int epre[kLabGroup + 1];
            epre[0] = 0;
#pragma unroll
            for (int j = 0; j < kLabGroup; ++j) epre[j + 1] = epre[j] + g.pre[j][8];
#pragma unroll 1
            for (int t = threadIdx.x; t < epre[kLabGroup]; t += kThreads) {
                int j, li;
                label_group_voxel(g, epre, t, j, li);
                my_votes += vote(g.slot[j], unpack_key(g.key[j]), li);
            }
            __syncthreads();  // the group's LDS is rewritten by the next group
        }
    } else {
        const int first = (int)blockIdx.x * (kThreads / 64) + wave, stride = (int)gridDim.x * (kThreads / 64);
        for (int e = first; e < n; e += stride) {
            const int slot = f.tk_slot[e];
            const int3 bc = unpack_key(f.tk_key[e]);
            const BandWords b = band_words(f, e);
#pragma unroll 1
            for (int t = lane; t < b.pre[8]; t += 64) my_votes += vote(slot, bc, band_select(b, t));
        }
    }
    const unsigned long long w = wave_sum_u64(my_votes);
    if (lane == 0) s_sum[wave] = w;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long t = 0;
        for (int i = 0; i < kThreads / 64; ++i) t += s_sum[i];
        if (t) spread_add(m.sync->votes, t);
    }
}

// Camera labels for every camera of the call, in order (equal to one call per camera: a
// voxel's votes are sequential): vote counts (kLatest false) or the latest label.
template <int kSched, bool kLatest>
__global__ __launch_bounds__(kThreads) void k_labels(MapView m, FrameView f, CameraSet cs)
{
    for_band_voxels<kSched>(m, f, [&](int slot, int3 bc, int li) {
        return kLatest ? label_voxel_latest(m, cs, slot, bc, li) : label_voxel(m, cs, slot, bc, li);
    });
}

// label fusion from a label range image under the scan model: a wavefront per touched
// block, its band voxels compacted
template <bool kLatest>
__global__ __launch_bounds__(kThreads) void k_labels_lidar(MapView m, FrameView f, LidarLUT L, Pose T,
                                                           const uint8_t *__restrict__ img)
{
    for_band_voxels<1>(m, f, [&](int slot, int3 bc, int li) {
        return label_voxel_lidar<kLatest>(m, L, T, img, slot, bc, li);
    });
}

// Eq. 6 on one camera's class log-probability image, over the band voxels of the last frame
__global__ __launch_bounds__(kThreads) void k_logprobs(MapView m, FrameView f, Camera cam, Pose T,
                                                       const float *__restrict__ logp)
{
    for_band_voxels<0>(m, f, [&](int slot, int3 bc, int li) { return logprob_voxel(m, cam, T, logp, slot, bc, li); });
}

hipError_t launch_labels_lidar(const MapView &m, const FrameView &f, const LidarLUT &lut, const Pose &T,
                               const uint8_t *img, int grid, int label_mode, hipStream_t s)
{
    if (label_mode == kLabelLatest)
        hipLaunchKernelGGL(k_labels_lidar<true>, dim3(grid), dim3(kThreads), 0, s, m, f, lut, T, img);
    else
        hipLaunchKernelGGL(k_labels_lidar<false>, dim3(grid), dim3(kThreads), 0, s, m, f, lut, T, img);
    return hipGetLastError();
}

hipError_t launch_labels(const MapView &m, const FrameView &f, const CameraSet &cams, int schedule, int grid,
                         int label_mode, hipStream_t s)
{
    const bool latest = label_mode == kLabelLatest;
    if (schedule == 0) {
        if (latest) hipLaunchKernelGGL((k_labels<0, true>), dim3(grid), dim3(kThreads), 0, s, m, f, cams);
        else hipLaunchKernelGGL((k_labels<0, false>), dim3(grid), dim3(kThreads), 0, s, m, f, cams);
    } else {
        if (latest) hipLaunchKernelGGL((k_labels<1, true>), dim3(grid), dim3(kThreads), 0, s, m, f, cams);
        else hipLaunchKernelGGL((k_labels<1, false>), dim3(grid), dim3(kThreads), 0, s, m, f, cams);
    }
    return hipGetLastError();
}

hipError_t launch_logprobs(const MapView &m, const FrameView &f, const Camera &cam, const Pose &T, const float *logp,
                           int grid, hipStream_t s)
{
    hipLaunchKernelGGL(k_logprobs, dim3(grid), dim3(kThreads), 0, s, m, f, cam, T, logp);
    return hipGetLastError();
}

}  // namespace mc
