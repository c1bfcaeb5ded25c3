// Marching cubes over the dirty (or all) blocks of one map: one workgroup per block (see
// mesh_device.h).  The triangle counter is parity-buffered: extraction p counts into
// tris[p] and clears tris[1 - p] (already read by the host) for the next one; the last
// workgroup clears the dirty set when a DIRTY extraction fit in the output.
#include "mesh_device.h"

namespace mc {

template <int kSched>
__global__ __launch_bounds__(kThreads) void k_mesh(MapView m, int mode, int parity, MeshOut out)
{
    // kSched 0: one workgroup per block; 1: one wavefront per block (own LDS region)
    constexpr size_t kLds = kSched == 0 ? sizeof(MeshLds) : (kThreads / 64) * sizeof(MeshLdsWave);
    __shared__ __align__(16) char smem[kLds];
    __shared__ int s_last;
    MeshLds &S = *reinterpret_cast<MeshLds *>(smem);
    MeshLdsWave *SW = reinterpret_cast<MeshLdsWave *>(smem);
    Counters *c = m.ctr;
    unsigned long long *tris = &c->tris[parity];
    const int nblk = mode == 0 ? c->n_dirty : c->pool_used;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        c->mesh_blocks = (unsigned long long)nblk;
        c->tris[1 - parity] = 0;
    }
    if (kSched == 0) {
        for (int e = blockIdx.x; e < nblk; e += gridDim.x)
            mesh_block(m, mode == 0 ? m.dirty_list[e] : e, out, tris, S);
    } else {
        const int wave = threadIdx.x >> 6;
        for (int e = blockIdx.x * (kThreads / 64) + wave; e < nblk; e += gridDim.x * (kThreads / 64))
            mesh_block_wave(m, mode == 0 ? m.dirty_list[e] : e, out, tris, SW[wave]);
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        wait_memory();  // every triangle reservation lands before the ticket
        s_last = atomicAdd(&c->mesh_done, 1u) == gridDim.x - 1;
    }
    __syncthreads();
    if (s_last && threadIdx.x == 0) {
        close_extraction(m, mode, tris, out.cap);
        c->mesh_done = 0;
    }
}

hipError_t launch_mesh(const MapView &m, int mode, int parity, const MeshOut &out, int schedule, int grid,
                       hipStream_t s)
{
    if (schedule == 0) hipLaunchKernelGGL(k_mesh<0>, dim3(grid), dim3(kThreads), 0, s, m, mode, parity, out);
    else hipLaunchKernelGGL(k_mesh<1>, dim3(grid), dim3(kThreads), 0, s, m, mode, parity, out);
    return hipGetLastError();
}

}  // namespace mc
