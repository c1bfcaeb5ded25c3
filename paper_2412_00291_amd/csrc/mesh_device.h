// Marching cubes of one 8^3 block by one workgroup (end of Sec. IV-C.3): the block and
// its +1 halo (9^3 voxels of distance, weight and fused label, ~6.6 KiB) are staged in
// LDS from up to eight blocks; each thread evaluates two cubes; a workgroup prefix sum of
// the per-cube triangle counts reserves one contiguous output range with one atomic.
#pragma once
#include "device.h"
#include "mc_table.inc"

namespace mc {

__device__ __forceinline__ void mesh_block(const MapView &m, int slot, const MeshOut &out,
                                           unsigned long long *tris, MeshLds &S)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const float nu = m.nu;
    const int4 bc = m.coords[slot];
    if (threadIdx.x < 8) {
        const int j = threadIdx.x;
        S.nb[j] = j == 0 ? slot : hash_find(m, pack_key(bc.x + (j & 1), bc.y + ((j >> 1) & 1), bc.z + ((j >> 2) & 1)));
    }
    __syncthreads();
    for (int h = threadIdx.x; h < kHaloVoxels; h += kThreads) {
        const int hx = h % kHalo, hy = (h / kHalo) % kHalo, hz = h / (kHalo * kHalo);
        const int j = (hx >> 3) | ((hy >> 3) << 1) | ((hz >> 3) << 2);
        const int s = S.nb[j];
        if (s >= 0) {
            const size_t vi = (size_t)s * kBlockVoxels + (hx & 7) + 8 * (hy & 7) + 64 * (hz & 7);
            S.dw[h] = m.dw[vi];
            S.fused[h] = m.fused[vi];
        } else {
            S.dw[h] = make_float2(0.0f, 0.0f);  // absent block: unobserved
            S.fused[h] = 255;
        }
    }
    __syncthreads();

    int mask[2], ntri[2];
#pragma unroll
    for (int it = 0; it < 2; ++it) {
        const int cube = it * kThreads + threadIdx.x;
        const int cx = cube & 7, cy = (cube >> 3) & 7, cz = cube >> 6;
        bool valid = true;
        int mk = 0;
#pragma unroll
        for (int n = 0; n < 8; ++n) {
            const float2 v = S.dw[halo_index(cx + (n & 1), cy + ((n >> 1) & 1), cz + ((n >> 2) & 1))];
            valid = valid && (v.y > 0.0f);
            mk |= (v.x < 0.0f ? 1 : 0) << n;
        }
        mask[it] = mk;
        ntri[it] = valid ? (int)MC_NTRI[mk] : 0;
    }
    // workgroup exclusive scan of the triangle counts
    const int mine = ntri[0] + ntri[1];
    int incl = mine;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int y = __shfl_up(incl, off, 64);
        if (lane >= off) incl += y;
    }
    if (lane == 63) S.wsum[wave] = incl;
    __syncthreads();
    if (threadIdx.x == 0) {
        int tot = 0;
        for (int w = 0; w < kThreads / 64; ++w) tot += S.wsum[w];
        S.base = tot ? atomicAdd(tris, (unsigned long long)tot) : 0ull;
    }
    __syncthreads();
    int woff = 0;
    for (int w = 0; w < wave; ++w) woff += S.wsum[w];
    long long t = (long long)S.base + woff + (incl - mine);
#pragma unroll
    for (int it = 0; it < 2; ++it) {
        const int cube = it * kThreads + threadIdx.x;
        const int cx = cube & 7, cy = (cube >> 3) & 7, cz = cube >> 6;
        for (int q = 0; q < ntri[it]; ++q, ++t) {
            if (t >= out.cap) continue;
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const int ed = MC_TRIS[mask[it]][3 * q + k];
                const int ax = ed >> 2;
                const int3 o = edge_base(ed);
                const int ax_ = cx + o.x, ay_ = cy + o.y, az_ = cz + o.z;
                const int ha = halo_index(ax_, ay_, az_);
                const int hb = halo_index(ax_ + (ax == 0), ay_ + (ax == 1), az_ + (ax == 2));
                const float Da = S.dw[ha].x, Db = S.dw[hb].x;
                const float tt = Da / (Da - Db);
                const int vx = 8 * bc.x + ax_, vy = 8 * bc.y + ay_, vz = 8 * bc.z + az_;
                float P[3] = {(float)vx * nu, (float)vy * nu, (float)vz * nu};
                P[ax] = P[ax] + tt * nu;
                float *dst = out.pos + (size_t)t * 9 + 3 * k;
                dst[0] = P[0];
                dst[1] = P[1];
                dst[2] = P[2];
                out.lab[(size_t)t * 3 + k] = fabsf(Da) <= fabsf(Db) ? S.fused[ha] : S.fused[hb];
                if (out.ekey) {
                    const long long off = 1LL << 19;
                    out.ekey[(size_t)t * 3 + k] = ((vx + off) << 42) | ((vy + off) << 22) | ((vz + off) << 2) | ax;
                }
            }
        }
    }
    __syncthreads();  // LDS reuse by the next block
}

// Close an extraction (one thread, after every worker has finished): clear the dirty set
// when a DIRTY extraction fit in the output.
__device__ __forceinline__ void close_extraction(const MapView &m, int mode, unsigned long long *tris, long long cap)
{
    const unsigned long long total = atomicAdd(tris, 0ull);
    if (mode == 0 && (long long)total <= cap) {
        m.ctr->n_dirty = 0;
        m.ctr->dirty_epoch += 1;
    }
}

}  // namespace mc

namespace mc {

// The same marching cubes of one block by one wavefront (8 cubes per lane), with the
// halo in the wavefront's own LDS region: four blocks in flight per workgroup.
struct MeshLdsWave {
    float2 dw[kHaloVoxels];
    uint8_t fused[kHaloVoxels];
    int nb[8];
};

__device__ __forceinline__ void wave_lds_sync() { __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront"); }

__device__ __forceinline__ void mesh_block_wave(const MapView &m, int slot, const MeshOut &out,
                                                unsigned long long *tris, MeshLdsWave &S)
{
    const int lane = threadIdx.x & 63;
    const float nu = m.nu;
    const int4 bc = m.coords[slot];
    if (lane < 8) {
        const int j = lane;
        S.nb[j] = j == 0 ? slot : hash_find(m, pack_key(bc.x + (j & 1), bc.y + ((j >> 1) & 1), bc.z + ((j >> 2) & 1)));
    }
    wave_lds_sync();
    for (int h = lane; h < kHaloVoxels; h += 64) {
        const int hx = h % kHalo, hy = (h / kHalo) % kHalo, hz = h / (kHalo * kHalo);
        const int j = (hx >> 3) | ((hy >> 3) << 1) | ((hz >> 3) << 2);
        const int s = S.nb[j];
        if (s >= 0) {
            const size_t vi = (size_t)s * kBlockVoxels + (hx & 7) + 8 * (hy & 7) + 64 * (hz & 7);
            S.dw[h] = m.dw[vi];
            S.fused[h] = m.fused[vi];
        } else {
            S.dw[h] = make_float2(0.0f, 0.0f);  // absent block: unobserved
            S.fused[h] = 255;
        }
    }
    wave_lds_sync();
    unsigned masks = 0;  // triangle counts of the lane's 8 cubes, 4 bits each
    int mine = 0;
    int mk8[8];
#pragma unroll
    for (int it = 0; it < 8; ++it) {
        const int cube = it * 64 + lane;
        const int cx = cube & 7, cy = (cube >> 3) & 7, cz = cube >> 6;
        bool valid = true;
        int mk = 0;
#pragma unroll
        for (int n = 0; n < 8; ++n) {
            const float2 v = S.dw[halo_index(cx + (n & 1), cy + ((n >> 1) & 1), cz + ((n >> 2) & 1))];
            valid = valid && (v.y > 0.0f);
            mk |= (v.x < 0.0f ? 1 : 0) << n;
        }
        const int nt = valid ? (int)MC_NTRI[mk] : 0;
        mk8[it] = mk;
        masks |= (unsigned)nt << (4 * it);
        mine += nt;
    }
    int incl = mine;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int y = __shfl_up(incl, off, 64);
        if (lane >= off) incl += y;
    }
    const int tot = __shfl(incl, 63, 64);
    unsigned long long base = 0;
    if (lane == 0 && tot) base = atomicAdd(tris, (unsigned long long)tot);
    base = __shfl(base, 0, 64);
    long long t = (long long)base + (incl - mine);
#pragma unroll
    for (int it = 0; it < 8; ++it) {
        const int cube = it * 64 + lane;
        const int cx = cube & 7, cy = (cube >> 3) & 7, cz = cube >> 6;
        const int nt = (masks >> (4 * it)) & 15;
        for (int q = 0; q < nt; ++q, ++t) {
            if (t >= out.cap) continue;
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const int ed = MC_TRIS[mk8[it]][3 * q + k];
                const int ax = ed >> 2;
                const int3 o = edge_base(ed);
                const int ax_ = cx + o.x, ay_ = cy + o.y, az_ = cz + o.z;
                const int ha = halo_index(ax_, ay_, az_);
                const int hb = halo_index(ax_ + (ax == 0), ay_ + (ax == 1), az_ + (ax == 2));
                const float Da = S.dw[ha].x, Db = S.dw[hb].x;
                const float tt = Da / (Da - Db);
                const int vx = 8 * bc.x + ax_, vy = 8 * bc.y + ay_, vz = 8 * bc.z + az_;
                float P[3] = {(float)vx * nu, (float)vy * nu, (float)vz * nu};
                P[ax] = P[ax] + tt * nu;
                float *dst = out.pos + (size_t)t * 9 + 3 * k;
                dst[0] = P[0];
                dst[1] = P[1];
                dst[2] = P[2];
                out.lab[(size_t)t * 3 + k] = fabsf(Da) <= fabsf(Db) ? S.fused[ha] : S.fused[hb];
                if (out.ekey) {
                    const long long off = 1LL << 19;
                    out.ekey[(size_t)t * 3 + k] = ((vx + off) << 42) | ((vy + off) << 22) | ((vz + off) << 2) | ax;
                }
            }
        }
    }
    wave_lds_sync();  // the halo is rewritten by the wave's next block
}

}  // namespace mc
