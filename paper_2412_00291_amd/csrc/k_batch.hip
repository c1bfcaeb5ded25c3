// Batched step over many maps of uneven size: one launch per phase (allocation, TSDF,
// labels, meshing) covers every map of the step, so a step is four launches (one graph
// launch when captured) instead of four per map.  Each phase's items (pixel tiles,
// touched entries, dirty blocks) are numbered across the maps by prefix sums, and the
// grid strides over them statically; each item runs the same device body as the
// per-map kernels, so every map ends bit-identical to its own plain calls.  The last
// workgroup of each phase does the per-map bookkeeping and lays out the next phase's
// prefix sums.
//
// Schedules for the TSDF and label phases: 0 = one workgroup per touched block (two
// voxels per thread), 1 = one wavefront per touched block (eight voxels per lane, four
// blocks in flight per workgroup).  The project's autotuner picks the schedule and grid.
#include "mesh_device.h"

namespace mc {

__device__ __forceinline__ int find_map(const int32_t *pre, int n, int i)
{
    int lo = 0, hi = n - 1;  // last map with pre[m] <= i
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (pre[mid] <= i) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

__device__ __forceinline__ bool last_of_grid(uint32_t *ticket, int *s_last)
{
    if (threadIdx.x == 0) {
        wait_memory();  // this workgroup's atomics land before its ticket
        *s_last = atomicAdd(ticket, 1u) == gridDim.x - 1;
    }
    __syncthreads();
    return *s_last;
}

// ---------------------------------------------------------------------------------
// allocation: the step's pixel tiles, each tile inside one map
// ---------------------------------------------------------------------------------

__global__ __launch_bounds__(kThreads) void k_batch_alloc(BatchMap *maps, BatchCtl *ctl, int n)
{
    __shared__ unsigned long long lk[kLdsKeys];
    __shared__ int s_tmp[kThreads / 64];
    __shared__ unsigned long long s_base;
    __shared__ int s_last;
    int mi = 0;
    while (mi + 1 < n && maps[mi + 1].tile0 <= (int)blockIdx.x) ++mi;
    const BatchMap &B = maps[mi];
    for (int i = threadIdx.x; i < kLdsKeys; i += kThreads) lk[i] = kEmpty;
    __syncthreads();
    const int pix = (blockIdx.x - B.tile0) * kThreads + threadIdx.x;
    if (pix < B.lut.rows * B.lut.cols) alloc_pixel(lk, B.v, B.f, B.lut, B.T, B.range, pix);
    __syncthreads();
    alloc_flush(lk, s_tmp, &s_base, B.v, B.f);
    if (last_of_grid(&ctl->done[0], &s_last) && threadIdx.x == 0) {
        int acc = 0;
        for (int m = 0; m < n; ++m) {
            const FrameState fs = frame_state(maps[m].v, maps[m].f);
            ctl->fs[m] = fs;
            ctl->pre_t[m] = acc;
            acc += fs.n_list;
        }
        ctl->pre_t[n] = acc;
        ctl->done[0] = 0;
    }
}

// ---------------------------------------------------------------------------------
// TSDF phase
// ---------------------------------------------------------------------------------

// Copy the prefix sums over maps into LDS (n + 1 entries).
__device__ __forceinline__ void load_prefix(int *dst, const int32_t *src, int n)
{
    for (int i = threadIdx.x; i <= n; i += kThreads) dst[i] = src[i];
    __syncthreads();
}

// Append this lane's dirty slot s (or nothing, s < 0) of map mi to that map's list; the
// wave's lanes may hold different maps, which are taken one map at a time.
__device__ __forceinline__ void dirty_append_maps(const BatchMap *maps, const BatchCtl *ctl, int mi, int s)
{
    unsigned long long pending = __ballot(s >= 0);
    while (pending) {
        const int leader = __ffsll((long long)pending) - 1;
        const int ml = __shfl(mi, leader, 64);
        const bool mine = s >= 0 && mi == ml;
        dirty_append_wave(maps[ml].v, mine ? s : -1, ctl->fs[ml].epoch);
        pending &= ~__ballot(mine);
    }
}

// Workers and chunks as in the per-map TSDF kernel, over the step's touched entries.
template <int kSched>
__global__ __launch_bounds__(kThreads) void k_batch_tsdf(BatchMap *maps, BatchCtl *ctl, int n)
{
    constexpr int kWidth = kSched == 0 ? kThreads : 64;
    constexpr int kChunk = kWidth / 8;
    __shared__ int s_pre[kMaxBatchMaps + 1];
    __shared__ int s_slot[kThreads / 8];
    __shared__ unsigned long long s_upd[kMaxBatchMaps];
    __shared__ int s_last;
    for (int i = threadIdx.x; i < kMaxBatchMaps; i += kThreads) s_upd[i] = 0;
    load_prefix(s_pre, ctl->pre_t, n);
    const int total = s_pre[n];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int rank = kSched == 0 ? (int)threadIdx.x : lane;
    const int first = kSched == 0 ? (int)blockIdx.x : (int)blockIdx.x * (kThreads / 64) + wave;
    const int stride = kSched == 0 ? (int)gridDim.x : (int)gridDim.x * (kThreads / 64);
    for (int base = first; base < total; base += kChunk * stride) {
        int my_slot = -1;
        const int ic = base + rank * stride;
        if (rank < kChunk && ic < total) {
            const int mi = find_map(s_pre, n, ic);
            const int e = ic - s_pre[mi];
            my_slot = commit_entry(maps[mi].v, maps[mi].f, ctl->fs[mi], e, maps[mi].f.tk_key[e], maps[mi].frame_id);
        }
        if (kSched == 0) {
            if (rank < kChunk) s_slot[rank] = my_slot;
            __syncthreads();
        }
        {
            const int i = rank >> 3;
            const int im = base + i * stride;
            const int si = kSched == 0 ? s_slot[i] : __shfl(my_slot, i, 64);
            int s = -1, mi = 0;
            if (im < total) {
                mi = find_map(s_pre, n, im);
                const int e = im - s_pre[mi];
                if (ctl->fs[mi].ok)
                    s = neighbour_slot(maps[mi].v, rank & 7, unpack_key(maps[mi].f.tk_key[e]), si, maps[mi].frame_id);
            }
            dirty_append_maps(maps, ctl, mi, s);
        }
        for (int j = 0; j < kChunk; ++j) {
            const int item = base + j * stride;
            if (item >= total) break;
            const int slot = kSched == 0 ? s_slot[j] : __shfl(my_slot, j, 64);
            const int mi = __builtin_amdgcn_readfirstlane(find_map(s_pre, n, item));  // uniform per worker
            if (!ctl->fs[mi].ok) continue;
            const BatchMap &B = maps[mi];
            const int e = item - s_pre[mi];
            unsigned long long upd = tsdf_block<kWidth>(B.v, B.f, B.lut, B.T, B.range, e, B.f.tk_key[e], slot, rank);
            upd = wave_sum_u64(upd);
            if (lane == 0 && upd) atomicAdd(&s_upd[mi], upd);
        }
        if (kSched == 0) __syncthreads();
    }
    __syncthreads();
    for (int m = threadIdx.x; m < n; m += kThreads)
        if (s_upd[m]) atomicAdd(&maps[m].v.ctr->updates, s_upd[m]);
    if (last_of_grid(&ctl->done[1], &s_last) && threadIdx.x == 0) {
        int acc_l = 0, acc_d = 0;
        for (int m = 0; m < n; ++m) {
            const BatchMap &B = maps[m];
            close_frame(B.v, frame_state(B.v, B.f));
            ctl->pre_l[m] = acc_l;
            acc_l += B.v.ctr->last_touched;
            ctl->pre_d[m] = acc_d;
            const int nd = coherent_load(&B.v.ctr->n_dirty);
            acc_d += nd;
            B.v.ctr->mesh_blocks = (unsigned long long)nd;
            B.v.ctr->tris[B.parity] = 0;
            B.v.ctr->tris[1 - B.parity] = 0;
        }
        ctl->pre_l[n] = acc_l;
        ctl->pre_d[n] = acc_d;
        ctl->done[1] = 0;
    }
}

// ---------------------------------------------------------------------------------
// label phase
// ---------------------------------------------------------------------------------

template <int kSched>
__global__ __launch_bounds__(kThreads) void k_batch_labels(BatchMap *maps, BatchCtl *ctl, int n)
{
    constexpr int kWidth = kSched == 0 ? kThreads : 64;
    __shared__ int s_pre[kMaxBatchMaps + 1];
    __shared__ unsigned long long s_votes[kMaxBatchMaps];
    for (int i = threadIdx.x; i < kMaxBatchMaps; i += kThreads) s_votes[i] = 0;
    load_prefix(s_pre, ctl->pre_l, n);
    const int total = s_pre[n];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int rank = kSched == 0 ? (int)threadIdx.x : lane;
    const int first = kSched == 0 ? (int)blockIdx.x : (int)blockIdx.x * (kThreads / 64) + wave;
    const int stride = kSched == 0 ? (int)gridDim.x : (int)gridDim.x * (kThreads / 64);
    for (int item = first; item < total; item += stride) {
        const int mi = __builtin_amdgcn_readfirstlane(find_map(s_pre, n, item));  // uniform per worker
        const BatchMap &B = maps[mi];
        if (B.cams.n == 0) continue;
        const int e = item - s_pre[mi];
        const int slot = B.f.tk_slot[e];
        const int3 bc = unpack_key(B.f.tk_key[e]);
        unsigned long long v = 0;
#pragma unroll
        for (int it = 0; it < kBlockVoxels / kWidth; ++it) {
            const int li = it * kWidth + rank;
            const unsigned long long bits = B.f.band[(size_t)e * 8 + (li >> 6)];
            if (bits == 0) continue;  // wave-uniform
            if ((bits >> (li & 63)) & 1ull) v += label_voxel(B.v, B.cams, slot, bc, li);
        }
        v = wave_sum_u64(v);
        if (lane == 0 && v) atomicAdd(&s_votes[mi], v);
    }
    __syncthreads();
    for (int m = threadIdx.x; m < n; m += kThreads)
        if (s_votes[m]) atomicAdd(&maps[m].v.ctr->votes, s_votes[m]);
}

// ---------------------------------------------------------------------------------
// meshing phase: one workgroup per dirty block
// ---------------------------------------------------------------------------------

__global__ __launch_bounds__(kThreads) void k_batch_mesh(BatchMap *maps, BatchCtl *ctl, int n)
{
    __shared__ MeshLds S;
    __shared__ int s_pre[kMaxBatchMaps + 1];
    __shared__ int s_last;
    load_prefix(s_pre, ctl->pre_d, n);
    const int total = s_pre[n];
    for (int item = blockIdx.x; item < total; item += gridDim.x) {
        const int mi = find_map(s_pre, n, item);
        const BatchMap &B = maps[mi];
        mesh_block(B.v, B.v.dirty_list[item - s_pre[mi]], B.out, &B.v.ctr->tris[B.parity], S);
    }
    if (last_of_grid(&ctl->done[3], &s_last) && threadIdx.x == 0) {
        for (int m = 0; m < n; ++m) {
            const BatchMap &B = maps[m];
            unsigned long long *tris = &B.v.ctr->tris[B.parity];
            close_extraction(B.v, 0, tris, B.out.cap);
            ctl->tris[m] = atomicAdd(tris, 0ull);
        }
        ctl->done[3] = 0;
    }
}

hipError_t launch_batch(BatchMap *maps, BatchCtl *ctl, int n_maps, int total_tiles, int schedule, int grid,
                        hipStream_t s)
{
    if (total_tiles > 0) hipLaunchKernelGGL(k_batch_alloc, dim3(total_tiles), dim3(kThreads), 0, s, maps, ctl, n_maps);
    else return hipErrorInvalidValue;
    if (schedule == 0) {
        hipLaunchKernelGGL(k_batch_tsdf<0>, dim3(grid), dim3(kThreads), 0, s, maps, ctl, n_maps);
        hipLaunchKernelGGL(k_batch_labels<0>, dim3(grid), dim3(kThreads), 0, s, maps, ctl, n_maps);
    } else {
        hipLaunchKernelGGL(k_batch_tsdf<1>, dim3(grid), dim3(kThreads), 0, s, maps, ctl, n_maps);
        hipLaunchKernelGGL(k_batch_labels<1>, dim3(grid), dim3(kThreads), 0, s, maps, ctl, n_maps);
    }
    hipLaunchKernelGGL(k_batch_mesh, dim3(grid), dim3(kThreads), 0, s, maps, ctl, n_maps);
    return hipGetLastError();
}

}  // namespace mc
