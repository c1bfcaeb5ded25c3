// Marching cubes over the dirty (or all) blocks of one map, in three launches: count
// triangles per workgroup, scan the counts (one workgroup, which also does the
// extraction's bookkeeping), emit at the scanned offsets.  Both passes take the same
// candidate blocks in the same order (see mesh_device.h), so the output is compact.
#include "mesh_device.h"

namespace mc {

__global__ __launch_bounds__(kThreads) void k_mesh_count(MapView m, int mode, MeshScan scan)
{
    __shared__ MeshSmem<1, HaloMask> S;
    const Counters *c = m.ctr;
    long long tris;
    int blocks;
    mesh_count_wg(m, mode != 0, c->dirty_epoch, c->pool_used, S, &tris, &blocks);
    if (threadIdx.x == 0) {
        scan.wg_tris[blockIdx.x] = tris;
        scan.wg_blocks[blockIdx.x] = blocks;
    }
}

__global__ __launch_bounds__(kThreads) void k_mesh_scan(MapView m, int mode, MeshScan scan, int G, int k, long long cap,
                                                        MeshReport *report)
{
    mesh_scan_map(m, mode, scan.wg_tris, scan.wg_blocks, scan.wg_off, G, k, 1, cap, report);
}

template <int kSched>
__global__ __launch_bounds__(kThreads) void k_mesh_emit(MapView m, int mode, MeshScan scan, MeshOut out)
{
    __shared__ MeshSmem<kSched, HaloFull> S;
    __shared__ MeshStage st;
    const Counters *c = m.ctr;
    mesh_emit_wg<kSched>(m, mode != 0, c->mesh_epoch, c->pool_used, scan.wg_off[blockIdx.x], out, S, st);
}

MeshGrid mesh_grid(int schedule)
{
    static MeshGrid cached[2] = {{0, 0}, {0, 0}};
    const int k = schedule != 0;
    if (!cached[k].emit)
        cached[k] = k == 0 ? resident_grids(k_mesh_count, k_mesh_emit<0>) : resident_grids(k_mesh_count, k_mesh_emit<1>);
    return cached[k];
}

hipError_t launch_mesh_count(const MapView &m, int mode, const MeshScan &scan, int schedule, MeshGrid grid,
                             hipStream_t s)
{
    if (grid.emit < 1 || grid.count < grid.emit || grid.count > kMaxMeshGrid || grid.count % grid.emit)
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_mesh_count, dim3(grid.count), dim3(kThreads), 0, s, m, mode, scan);
    return hipGetLastError();
}

hipError_t launch_mesh_finish(const MapView &m, int mode, const MeshOut &out, const MeshScan &scan,
                              MeshReport *report, int schedule, MeshGrid grid, hipStream_t s)
{
    if (grid.emit < 1 || grid.count < grid.emit || grid.count > kMaxMeshGrid || grid.count % grid.emit)
        return hipErrorInvalidValue;
    const int k = grid.count / grid.emit;
    hipLaunchKernelGGL(k_mesh_scan, dim3(1), dim3(kThreads), 0, s, m, mode, scan, grid.emit, k, out.cap, report);
    if (schedule == 0) hipLaunchKernelGGL(k_mesh_emit<0>, dim3(grid.emit), dim3(kThreads), 0, s, m, mode, scan, out);
    else hipLaunchKernelGGL(k_mesh_emit<1>, dim3(grid.emit), dim3(kThreads), 0, s, m, mode, scan, out);
    return hipGetLastError();
}

}  // namespace mc
