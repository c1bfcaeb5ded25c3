// Marching cubes over the dirty (or all) blocks of one map: one workgroup per block (see
// mesh_device.h).  The triangle counter is parity-buffered: extraction p counts into
// tris[p] and clears tris[1 - p] (already read by the host) for the next one; the last
// workgroup clears the dirty set when a DIRTY extraction fit in the output.
#include "mesh_device.h"

namespace mc {

__global__ __launch_bounds__(kThreads) void k_mesh(MapView m, int mode, int parity, MeshOut out)
{
    __shared__ MeshLds S;
    __shared__ int s_last;
    Counters *c = m.ctr;
    unsigned long long *tris = &c->tris[parity];
    const int nblk = mode == 0 ? c->n_dirty : c->pool_used;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        c->mesh_blocks = (unsigned long long)nblk;
        c->tris[1 - parity] = 0;
    }
    for (int e = blockIdx.x; e < nblk; e += gridDim.x)
        mesh_block(m, mode == 0 ? m.dirty_list[e] : e, out, tris, S);
    if (threadIdx.x == 0) {
        __threadfence();
        s_last = atomicAdd(&c->mesh_done, 1u) == gridDim.x - 1;
    }
    __syncthreads();
    if (s_last && threadIdx.x == 0) {
        __threadfence();
        close_extraction(m, mode, tris, out.cap);
        c->mesh_done = 0;
    }
}

hipError_t launch_mesh(const MapView &m, int mode, int parity, const MeshOut &out, int grid, hipStream_t s)
{
    hipLaunchKernelGGL(k_mesh, dim3(grid), dim3(kThreads), 0, s, m, mode, parity, out);
    return hipGetLastError();
}

}  // namespace mc
