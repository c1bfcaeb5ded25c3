// Batched step over many maps of uneven size: one launch per phase (allocation, TSDF,
// labels, meshing) covers every map of the step, so a step is four launches (one graph
// launch when captured) instead of four per map.  Workgroups pull (map, item) pairs from
// device queues laid out by prefix sums over the maps; each item runs the same device
// body as the per-map kernels, so every map ends bit-identical to its own plain calls.
// The last workgroup of each phase does the per-map bookkeeping and lays out the next
// phase's queue.
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
            ctl->pre_t[m] = acc;
            acc += frame_state(maps[m].v, maps[m].f).n_list;
        }
        ctl->pre_t[n] = acc;
        ctl->queue[0] = 0;
        ctl->done[0] = 0;
    }
}

// ---------------------------------------------------------------------------------
// TSDF phase
// ---------------------------------------------------------------------------------

template <int kSched>
__global__ __launch_bounds__(kThreads) void k_batch_tsdf(BatchMap *maps, BatchCtl *ctl, int n)
{
    __shared__ int s_item[1];
    __shared__ int s_slot[1];
    __shared__ unsigned long long s_upd[kMaxBatchMaps];
    __shared__ int s_last;
    for (int i = threadIdx.x; i < kMaxBatchMaps; i += kThreads) s_upd[i] = 0;
    __syncthreads();
    const int total = ctl->pre_t[n];
    const int lane = threadIdx.x & 63;
    // kSched 0: the workgroup takes one item at a time; 1: each wave takes its own
    for (;;) {
        int item = 0;
        if (kSched == 0) {
            if (threadIdx.x == 0) s_item[0] = (int)atomicAdd(&ctl->queue[0], 1u);
            __syncthreads();
            item = s_item[0];
        } else {
            if (lane == 0) item = (int)atomicAdd(&ctl->queue[0], 1u);
            item = __shfl(item, 0, 64);
        }
        if (item >= total) break;
        const int mi = find_map(ctl->pre_t, n, item);
        const int e = item - ctl->pre_t[mi];
        const BatchMap &B = maps[mi];
        const FrameState fs = frame_state(B.v, B.f);
        const unsigned long long key = B.f.tk_key[e];
        int slot = 0;
        if (kSched == 0) {
            if (threadIdx.x == 0) s_slot[0] = commit_entry(B.v, B.f, fs, e, key, B.frame_id);
            __syncthreads();
            slot = s_slot[0];
        } else {
            if (lane == 0) slot = commit_entry(B.v, B.f, fs, e, key, B.frame_id);
            slot = __shfl(slot, 0, 64);
        }
        if (fs.ok) {
            const int3 bc = unpack_key(key);
            const int rank = kSched == 0 ? (int)threadIdx.x : lane;
            if (rank < 8) mark_neighbours(B.v, rank, bc, slot, fs.epoch, B.frame_id);
            float2 *dwb = B.v.dw + (size_t)slot * kBlockVoxels;
            unsigned long long upd = 0;
            constexpr int kWidth = kSched == 0 ? kThreads : 64;
#pragma unroll
            for (int it = 0; it < kBlockVoxels / kWidth; ++it) {
                const int li = it * kWidth + rank;
                bool band;
                upd += tsdf_voxel(B.v, B.lut, B.T, B.range, dwb, bc, li, band);
                const unsigned long long bits = __ballot(band);
                if (lane == 0) B.f.band[(size_t)e * 8 + (li >> 6)] = bits;
            }
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
        ctl->queue[1] = 0;
        ctl->queue[2] = 0;
        ctl->done[1] = 0;
    }
}

// ---------------------------------------------------------------------------------
// label phase
// ---------------------------------------------------------------------------------

template <int kSched>
__global__ __launch_bounds__(kThreads) void k_batch_labels(BatchMap *maps, BatchCtl *ctl, int n)
{
    __shared__ int s_item[1];
    __shared__ unsigned long long s_votes[kMaxBatchMaps];
    for (int i = threadIdx.x; i < kMaxBatchMaps; i += kThreads) s_votes[i] = 0;
    __syncthreads();
    const int total = ctl->pre_l[n];
    const int lane = threadIdx.x & 63;
    for (;;) {
        int item = 0;
        if (kSched == 0) {
            if (threadIdx.x == 0) s_item[0] = (int)atomicAdd(&ctl->queue[1], 1u);
            __syncthreads();
            item = s_item[0];
            __syncthreads();  // s_item is rewritten by the next take
        } else {
            if (lane == 0) item = (int)atomicAdd(&ctl->queue[1], 1u);
            item = __shfl(item, 0, 64);
        }
        if (item >= total) break;
        const int mi = find_map(ctl->pre_l, n, item);
        const int e = item - ctl->pre_l[mi];
        const BatchMap &B = maps[mi];
        if (B.cams.n == 0) continue;
        const int slot = B.f.tk_slot[e];
        const int3 bc = unpack_key(B.f.tk_key[e]);
        constexpr int kWidth = kSched == 0 ? kThreads : 64;
        const int rank = kSched == 0 ? (int)threadIdx.x : lane;
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
    __shared__ int s_item;
    __shared__ int s_last;
    const int total = ctl->pre_d[n];
    for (;;) {
        if (threadIdx.x == 0) s_item = (int)atomicAdd(&ctl->queue[2], 1u);
        __syncthreads();
        const int item = s_item;
        __syncthreads();
        if (item >= total) break;
        const int mi = find_map(ctl->pre_d, n, item);
        const BatchMap &B = maps[mi];
        mesh_block(B.v, B.v.dirty_list[item - ctl->pre_d[mi]], B.out, &B.v.ctr->tris[B.parity], S);
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
