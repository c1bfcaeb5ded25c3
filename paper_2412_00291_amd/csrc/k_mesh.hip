// Marching cubes over whole 8^3 blocks (end of Sec. IV-C.3).  One workgroup per block:
// the block and its +1 halo (9^3 voxels of distance, weight and fused label, ~6.6 KiB)
// are staged in LDS from up to eight blocks; each thread evaluates two cubes, a
// workgroup prefix sum of the per-cube triangle counts reserves one contiguous output
// range with a single atomic, and every thread writes its triangles there.
#include "internal.h"
#include "mc_table.inc"

namespace mc {

constexpr int kThreads = 256;
constexpr int kHalo = 9;
constexpr int kHaloVoxels = kHalo * kHalo * kHalo;

__global__ void k_mesh_begin(Counters *c)
{
    c->tris = 0;
    c->mesh_blocks = 0;
}

__global__ void k_mesh_end(Counters *c)
{
    c->n_dirty = 0;
    c->dirty_epoch += 1;
}

hipError_t launch_mesh_begin(const MapView &m, hipStream_t s)
{
    hipLaunchKernelGGL(k_mesh_begin, dim3(1), dim3(1), 0, s, m.ctr);
    return hipGetLastError();
}

hipError_t launch_mesh_end(const MapView &m, hipStream_t s)
{
    hipLaunchKernelGGL(k_mesh_end, dim3(1), dim3(1), 0, s, m.ctr);
    return hipGetLastError();
}

__device__ __forceinline__ int halo_index(int x, int y, int z) { return x + kHalo * (y + kHalo * z); }

// local base corner of cube edge e (axis e / 4, the other two offsets from e % 4)
__device__ __forceinline__ int3 edge_base(int e)
{
    const int ax = e >> 2, j = e & 3;
    if (ax == 0) return make_int3(0, j & 1, j >> 1);
    if (ax == 1) return make_int3(j & 1, 0, j >> 1);
    return make_int3(j & 1, j >> 1, 0);
}

__global__ __launch_bounds__(kThreads) void k_mesh(MapView m, int mode, MeshOut out)
{
    __shared__ float2 sdw[kHaloVoxels];
    __shared__ uint8_t sf[kHaloVoxels];
    __shared__ int snb[8];
    __shared__ int s_wsum[kThreads / 64];
    __shared__ unsigned long long s_base;
    Counters *c = m.ctr;
    const int nblk = mode == 0 ? c->n_dirty : c->pool_used;
    if (blockIdx.x == 0 && threadIdx.x == 0) c->mesh_blocks = (unsigned long long)nblk;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const float nu = m.nu;
    for (int e = blockIdx.x; e < nblk; e += gridDim.x) {
        const int slot = mode == 0 ? m.dirty_list[e] : e;
        const int4 bc = m.coords[slot];
        if (threadIdx.x < 8) {
            const int j = threadIdx.x;
            snb[j] = j == 0 ? slot
                            : hash_find(m, pack_key(bc.x + (j & 1), bc.y + ((j >> 1) & 1), bc.z + ((j >> 2) & 1)));
        }
        __syncthreads();
        for (int h = threadIdx.x; h < kHaloVoxels; h += kThreads) {
            const int hx = h % kHalo, hy = (h / kHalo) % kHalo, hz = h / (kHalo * kHalo);
            const int j = (hx >> 3) | ((hy >> 3) << 1) | ((hz >> 3) << 2);
            const int s = snb[j];
            if (s >= 0) {
                const size_t vi = (size_t)s * kBlockVoxels + (hx & 7) + 8 * (hy & 7) + 64 * (hz & 7);
                sdw[h] = m.dw[vi];
                sf[h] = m.fused[vi];
            } else {
                sdw[h] = make_float2(0.0f, 0.0f);  // absent block: unobserved
                sf[h] = 255;
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
                const float2 v = sdw[halo_index(cx + (n & 1), cy + ((n >> 1) & 1), cz + ((n >> 2) & 1))];
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
        if (lane == 63) s_wsum[wave] = incl;
        __syncthreads();
        if (threadIdx.x == 0) {
            int tot = 0;
            for (int w = 0; w < kThreads / 64; ++w) tot += s_wsum[w];
            s_base = tot ? atomicAdd(&c->tris, (unsigned long long)tot) : 0ull;
        }
        __syncthreads();
        int woff = 0;
        for (int w = 0; w < wave; ++w) woff += s_wsum[w];
        long long t = (long long)s_base + woff + (incl - mine);
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
                    const float Da = sdw[ha].x, Db = sdw[hb].x;
                    const float tt = Da / (Da - Db);
                    const int vx = 8 * bc.x + ax_, vy = 8 * bc.y + ay_, vz = 8 * bc.z + az_;
                    float P[3] = {(float)vx * nu, (float)vy * nu, (float)vz * nu};
                    P[ax] = P[ax] + tt * nu;
                    float *dst = out.pos + (size_t)t * 9 + 3 * k;
                    dst[0] = P[0];
                    dst[1] = P[1];
                    dst[2] = P[2];
                    out.lab[(size_t)t * 3 + k] = fabsf(Da) <= fabsf(Db) ? sf[ha] : sf[hb];
                    if (out.ekey) {
                        const long long off = 1LL << 19;
                        out.ekey[(size_t)t * 3 + k] = ((vx + off) << 42) | ((vy + off) << 22) | ((vz + off) << 2) | ax;
                    }
                }
            }
        }
        __syncthreads();  // LDS reuse by the next block
    }
}

hipError_t launch_mesh(const MapView &m, int mode, const MeshOut &out, int grid, hipStream_t s)
{
    hipLaunchKernelGGL(k_mesh, dim3(grid), dim3(kThreads), 0, s, m, mode, out);
    return hipGetLastError();
}

}  // namespace mc
