// Batched step over many maps of uneven size: one launch per phase (allocation, TSDF,
// labels, meshing in three passes) covers every map of the step, so a step is six
// launches (one graph launch when captured) instead of six per map.  Each phase's items
// (pixel tiles, touched entries, mesh candidates) are numbered across the maps by prefix
// sums, and the grid strides over them statically; each item runs the same device body
// as the per-map kernels, so every map ends bit-identical to its own plain calls.  The
// last workgroup of the allocation and TSDF phases (hierarchical tickets) does the
// per-map bookkeeping and lays out the next phase's prefix sums.
//
// Schedules for the TSDF and label phases (bit 0 and bit 1 of the schedule): 0 = one
// workgroup per touched block (two voxels per thread), 1 = one wavefront per touched block
// (eight voxels per lane, four blocks in flight per workgroup).  Meshing uses one wavefront
// per block.  The project's autotuner picks the schedules and the grid.
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

// ---------------------------------------------------------------------------------
// allocation: the step's pixel tiles, each tile inside one map
// ---------------------------------------------------------------------------------

__global__ __launch_bounds__(kThreads) void k_batch_alloc(BatchMap *maps, BatchCtl *ctl, BatchSync *sync, int n)
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
    if (threadIdx.x == 0) s_last = ticket_arrive(sync->alloc);
    __syncthreads();
    if (s_last && threadIdx.x == 0) {
        int acc = 0;
        for (int m = 0; m < n; ++m) {
            const FrameState fs = frame_state_coherent(maps[m].v, maps[m].f);
            ctl->fs[m] = fs;
            ctl->pre_t[m] = acc;
            acc += fs.n_list;
        }
        ctl->pre_t[n] = acc;
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

// Workers and chunks as in the per-map TSDF kernel, over the step's touched entries.
template <int kSched>
__global__ __launch_bounds__(kThreads) void k_batch_tsdf(BatchMap *maps, BatchCtl *ctl, BatchSync *sync, int n)
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
        {  // dirty marks last, as in the per-map kernel
            const int i = rank >> 3;
            const int im = base + i * stride;
            const int si = kSched == 0 ? s_slot[i] : __shfl(my_slot, i, 64);
            if (im < total) {
                const int mi = find_map(s_pre, n, im);
                const int e = im - s_pre[mi];
                const FrameState &fs = ctl->fs[mi];
                if (fs.ok) {
                    const MapView &v = maps[mi].v;
                    const int s = neighbour_slot(v, rank & 7, unpack_key(maps[mi].f.tk_key[e]), si, maps[mi].frame_id);
                    if (s >= 0) mark_dirty(v, s, fs.epoch, fs.bits);
                }
            }
        }
        if (kSched == 0) __syncthreads();
    }
    __syncthreads();
    for (int m = threadIdx.x; m < n; m += kThreads)
        if (s_upd[m]) spread_add(maps[m].v.sync->updates, s_upd[m]);
    if (threadIdx.x == 0) s_last = ticket_arrive(sync->tsdf);
    __syncthreads();
    if (!s_last) return;
    for (int m = wave; m < n; m += kThreads / 64) close_frame_wave(maps[m].v, ctl->fs[m]);
    if (threadIdx.x == 0) {
        int acc_l = 0, acc_p = 0;
        for (int m = 0; m < n; ++m) {
            const FrameState &fs = ctl->fs[m];
            ctl->pre_l[m] = acc_l;
            acc_l += fs.ok ? fs.n_list : 0;
            ctl->pre_p[m] = acc_p;
            acc_p += fs.ok ? fs.used + fs.n_new : fs.used;
        }
        ctl->pre_l[n] = acc_l;
        ctl->pre_p[n] = acc_p;
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
        const BandWords bw = band_words(B.f, e);
        for (int t = rank; t < bw.pre[8]; t += kWidth) v += label_voxel(B.v, B.cams, slot, bc, band_select(bw, t));
        v = wave_sum_u64(v);
        if (lane == 0 && v) atomicAdd(&s_votes[mi], v);
    }
    __syncthreads();
    for (int m = threadIdx.x; m < n; m += kThreads)
        if (s_votes[m]) spread_add(maps[m].v.sync->votes, s_votes[m]);
}

// ---------------------------------------------------------------------------------
// meshing phase: counting pass, per-map scans, emitting pass (one workgroup per block)
// ---------------------------------------------------------------------------------

// One iteration's candidates of this workgroup over the step's concatenated pool slots
// (map m's slots are items pre[m] .. pre[m+1]-1), compacted into S.list as item numbers;
// dealt out as in the per-map passes.  Returns their number, or -1 past the end.
template <class Smem>
__device__ __forceinline__ int batch_candidates(const BatchMap *maps, const int *s_pre, const uint32_t *s_epoch,
                                                int n, int it, bool need_tris, Smem &S)
{
    const int total = s_pre[n];
    if (((long long)it * kThreads * gridDim.x + blockIdx.x) >= total) return -1;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const long long item = ((long long)it * kThreads + threadIdx.x) * gridDim.x + blockIdx.x;
    bool take = false;
    if (item < total) {
        const int mi = find_map(s_pre, n, (int)item);
        const MapView &v = maps[mi].v;
        const bool dirty = is_dirty(v, item - s_pre[mi], s_epoch[mi]);
        const uint16_t nt = need_tris ? v.mesh_cnt[item - s_pre[mi]] : (uint16_t)1;
        take = dirty && nt != 0;
    }
    const unsigned long long bal = __ballot(take);
    if (lane == 0) S.wcnt[wave] = __popcll(bal);
    __syncthreads();
    int off = 0, cnt = 0;
#pragma unroll
    for (int w = 0; w < kThreads / 64; ++w) {
        const int c = S.wcnt[w];
        off += w < wave ? c : 0;
        cnt += c;
    }
    if (take) S.list[off + __popcll(bal & ((1ull << lane) - 1ull))] = (int)item;
    __syncthreads();
    return cnt;
}

// Map, coordinates and neighbour slots of list entries j0 .. j0 + nb - 1 (as
// mesh_batch_lookup, the map resolved per entry).
template <class Smem>
__device__ __forceinline__ void batch_lookup(const BatchMap *maps, const int *s_pre, int n, Smem &S, int j0, int nb,
                                             bool fetch)
{
    const int jb = threadIdx.x >> 3, e = threadIdx.x & 7;
    if (jb < nb) {
        const int item = S.list[j0 + jb];
        const int mi = find_map(s_pre, n, item);
        const MapView &v = maps[mi].v;
        const int slot = item - s_pre[mi];
        int s;
        if (fetch) {
            s = v.mesh_nbr[(size_t)slot * 8 + e];
            if (e == 0) S.bcs[jb] = v.coords[slot];
        } else {
            const int4 bc = v.coords[slot];
            if (e == 0) S.bcs[jb] = make_int4(bc.x, bc.y, bc.z, 0);  // .w unused: not read
            s = e == 0 ? slot : hash_find(v, pack_key(bc.x + (e & 1), bc.y + ((e >> 1) & 1), bc.z + ((e >> 2) & 1)));
            v.mesh_nbr[(size_t)slot * 8 + e] = s;
        }
        if (e == 0) S.mis[jb] = mi;
        S.nbs[jb][e] = s;
    }
    __syncthreads();
}

// One wavefront per block, four blocks in flight per workgroup (as the per-map passes'
// wavefront schedule); per-map totals are summed in LDS.
__global__ __launch_bounds__(kThreads) void k_batch_mesh_count(BatchMap *maps, BatchCtl *ctl, MeshScan scan, int n)
{
    __shared__ MeshSmem<1, HaloMask> S;
    __shared__ int s_pre[kMaxBatchMaps + 1];
    __shared__ uint32_t s_epoch[kMaxBatchMaps];
    __shared__ unsigned long long s_tris[kMaxBatchMaps];
    __shared__ unsigned s_blocks[kMaxBatchMaps];
    for (int m = threadIdx.x; m < n; m += kThreads) {
        s_epoch[m] = maps[m].v.ctr->dirty_epoch;
        s_tris[m] = 0;
        s_blocks[m] = 0;
    }
    load_prefix(s_pre, ctl->pre_p, n);
    const TableRegs tab = mesh_tables_load<false>();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    unsigned counts;
    for (int it = 0;; ++it) {
        const int cnt = batch_candidates(maps, s_pre, s_epoch, n, it, false, S);
        if (it == 0) mesh_tables_store<false>(S, tab);
        if (cnt < 0) break;
        for (int j0 = 0; j0 < cnt; j0 += kMeshBatch) {
            const int nb = cnt - j0 < kMeshBatch ? cnt - j0 : kMeshBatch;
            batch_lookup(maps, s_pre, n, S, j0, nb, false);
            for (int j = wave; j < nb; j += kThreads / 64) {
                const int mi = S.mis[j];
                mesh_stage_masks(maps[mi].v, S.nbs[j], S.h[wave], lane);
                const unsigned long long t =
                    wave_sum_u64((unsigned long long)mesh_classify_rows(S.h[wave], S.ntri, lane, nullptr, &counts));
                wave_lds_sync();
                if (lane == 0) {
                    maps[mi].v.mesh_cnt[S.nbs[j][0]] = (uint16_t)t;
                    atomicAdd(&s_tris[mi], t);
                    atomicAdd(&s_blocks[mi], 1u);
                }
            }
            __syncthreads();  // the batch's lookups are rewritten by the next batch
        }
        __syncthreads();
    }
    for (int m = threadIdx.x; m < n; m += kThreads) {
        scan.wg_tris[(size_t)blockIdx.x * n + m] = (long long)s_tris[m];
        scan.wg_blocks[(size_t)blockIdx.x * n + m] = (int)s_blocks[m];
    }
}

// One workgroup per map: that map's offsets over the counting pass's workgroups.
__global__ __launch_bounds__(kThreads) void k_batch_mesh_scan(BatchMap *maps, MeshScan scan, MeshReport *reports, int n,
                                                              int G, int k)
{
    const int m = blockIdx.x;
    const BatchMap &B = maps[m];
    mesh_scan_map(B.v, 0, scan.wg_tris + m, scan.wg_blocks + m, scan.wg_off + m, G, k, n, B.out.cap, &reports[m]);
}

// One wavefront per block; a round takes up to four consecutive candidates of one map
// (the list is in item order, so a map's blocks are consecutive), so that the round's
// output is one contiguous range of that map's buffer.
__global__ __launch_bounds__(kThreads) void k_batch_mesh_emit(BatchMap *maps, BatchCtl *ctl, MeshScan scan, int n)
{
    __shared__ MeshSmem<1, HaloFull> S;
    __shared__ MeshStage st;
    __shared__ int s_pre[kMaxBatchMaps + 1];
    __shared__ uint32_t s_epoch[kMaxBatchMaps];
    __shared__ long long s_next[kMaxBatchMaps];
    for (int m = threadIdx.x; m < n; m += kThreads) {
        s_epoch[m] = maps[m].v.ctr->mesh_epoch;
        s_next[m] = scan.wg_off[(size_t)blockIdx.x * n + m];
    }
    load_prefix(s_pre, ctl->pre_p, n);
    const TableRegs tab = mesh_tables_load<true>();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    unsigned counts = 0;
    for (int it = 0;; ++it) {
        const int cnt = batch_candidates(maps, s_pre, s_epoch, n, it, true, S);
        if (it == 0) mesh_tables_store<true>(S, tab);
        if (cnt < 0) break;
        for (int j0 = 0; j0 < cnt; j0 += kMeshBatch) {
            const int nb = cnt - j0 < kMeshBatch ? cnt - j0 : kMeshBatch;
            batch_lookup(maps, s_pre, n, S, j0, nb, true);
            for (int r = 0; r < nb;) {
                const int mr = S.mis[r];
                int in_round = 1;
                while (in_round < kThreads / 64 && r + in_round < nb && S.mis[r + in_round] == mr) ++in_round;
                const int j = r + wave;
                const bool has = wave < in_round;
                const BatchMap &B = maps[mr];
                int mine = 0;
                if (has) {
                    mesh_stage_rows(B.v, S.nbs[j], S.h[wave], lane);
                    if (lane == 0) S.rbc[wave] = S.bcs[j];
                    mine = mesh_classify_rows(S.h[wave], S.ntri, lane, S.ccase[wave], &counts);
                }
                const int incl = wave_scan_incl(mine);
                if (lane == 63) S.rcnt[wave] = incl;
                __syncthreads();
                int woff = 0, rtot = 0;
#pragma unroll
                for (int w = 0; w < kThreads / 64; ++w) {
                    const int c = (int)S.rcnt[w];
                    woff += w < wave ? c : 0;
                    rtot += c;
                }
                const long long r0 = s_next[mr];
                mesh_round_out<1>(B.v, S, st, has, counts, woff + incl - mine, rtot, r0, B.out);
                __syncthreads();  // every thread has read s_next[mr] and the round's counts
                if (threadIdx.x == 0) s_next[mr] = r0 + rtot;
                __syncthreads();
                r += in_round;
            }
        }
        __syncthreads();
    }
}

MeshGrid batch_mesh_grid()
{
    static MeshGrid cached = {0, 0};
    if (!cached.emit) cached = resident_grids(k_batch_mesh_count, k_batch_mesh_emit);
    return cached;
}

hipError_t launch_batch(BatchMap *maps, BatchCtl *ctl, BatchSync *sync, MeshScan scan, MeshReport *reports,
                        int n_maps, int total_tiles, int schedule, int grid, hipStream_t s)
{
    const MeshGrid mg = batch_mesh_grid();
    if (total_tiles < 1 || grid < 1 || grid > kMaxMeshGrid) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_batch_alloc, dim3(total_tiles), dim3(kThreads), 0, s, maps, ctl, sync, n_maps);
    if ((schedule & 1) == 0) hipLaunchKernelGGL(k_batch_tsdf<0>, dim3(grid), dim3(kThreads), 0, s, maps, ctl, sync, n_maps);
    else hipLaunchKernelGGL(k_batch_tsdf<1>, dim3(grid), dim3(kThreads), 0, s, maps, ctl, sync, n_maps);
    if ((schedule & 2) == 0) hipLaunchKernelGGL(k_batch_labels<0>, dim3(grid), dim3(kThreads), 0, s, maps, ctl, n_maps);
    else hipLaunchKernelGGL(k_batch_labels<1>, dim3(grid), dim3(kThreads), 0, s, maps, ctl, n_maps);
    hipLaunchKernelGGL(k_batch_mesh_count, dim3(mg.count), dim3(kThreads), 0, s, maps, ctl, scan, n_maps);
    hipLaunchKernelGGL(k_batch_mesh_scan, dim3(n_maps), dim3(kThreads), 0, s, maps, scan, reports, n_maps, mg.emit,
                       mg.count / mg.emit);
    hipLaunchKernelGGL(k_batch_mesh_emit, dim3(mg.emit), dim3(kThreads), 0, s, maps, ctl, scan, n_maps);
    return hipGetLastError();
}

}  // namespace mc
