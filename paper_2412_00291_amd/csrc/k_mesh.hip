// Marching cubes over the dirty (or all) blocks of one map, in two launches: count
// triangles per workgroup and record the blocks with triangles, then emit from those
// records, each emitting workgroup at the sum of the counts before it (workgroup 0 also
// does the extraction's bookkeeping and the host report).  The emitting workgroup takes
// its counting workgroups' records in their order, so the output is compact.
#include "mesh_device.h"

namespace mc {

// A DIRTY extraction takes its candidates from the dirty bitmap (and clears it) when the
// map holds more than bits_from blocks, every frame since the bitmap was last cleared has
// marked it, the bitmap is laid out for this grid and the host allows it (allow_bits: no
// change of layout since the last DIRTY extraction); otherwise it sweeps the slots.
__global__ __launch_bounds__(kThreads, 8) void k_mesh_count(MapView m, int mode, MeshScan scan, int allow_bits)
{
    __shared__ MeshSmem<1, HaloMask> S;
    const Counters *c = m.ctr;
    const uint32_t epoch = c->dirty_epoch;
    const int nslots = c->pool_used;
    const bool bits = mode == 0 && allow_bits && c->bits_gap == 0 && nslots > m.bits_from &&
                      (int)gridDim.x == m.bits_grid && (long long)nslots <= (long long)kThreads * 32 * gridDim.x;
    long long tris;
    int blocks;
    mesh_count_wg(m, mode != 0, epoch, nslots, S, &tris, &blocks, scan.rec + (size_t)blockIdx.x * scan.rec_cap,
                  scan.wg_nz + blockIdx.x, scan.rec_cap, bits);
    if (threadIdx.x == 0) {
        scan.wg_tris[blockIdx.x] = tris;
        scan.wg_blocks[blockIdx.x] = blocks;
        if (blockIdx.x == 0) {
            m.ctr->mesh_epoch = epoch;  // the emitting pass meshes this epoch
            m.ctr->mesh_bits = bits;
        }
    }
}

template <int kSched>
__global__ __launch_bounds__(kThreads) void k_mesh_emit(MapView m, int mode, MeshScan scan, MeshOut out, int g_count,
                                                       MeshReport *report)
{
    __shared__ MeshSmem<kSched, HaloFull> S;
    __shared__ MeshStage st;
    __shared__ long long s_red[3 * (kThreads / 64)];
    const TableRegs tab = mesh_tables_load<true>();  // in flight with the counts
    const int k = g_count / (int)gridDim.x;
    // the record counts of this workgroup's counting workgroups, also in flight with the counts
    const int my_nz = threadIdx.x < k ? scan.wg_nz[blockIdx.x + threadIdx.x * gridDim.x] : 0;
    const long long base = mesh_emit_base(m, mode, scan.wg_tris, scan.wg_blocks, g_count, out.cap, report, s_red);
    mesh_emit_recs<kSched>(m, scan, k, my_nz, base, out, S, st, tab);
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
                             bool allow_bits, hipStream_t s)
{
    if (grid.emit < 1 || grid.count < grid.emit || grid.count > kMaxMeshGrid || grid.count % grid.emit)
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_mesh_count, dim3(grid.count), dim3(kThreads), 0, s, m, mode, scan, (int)allow_bits);
    return hipGetLastError();
}

hipError_t launch_mesh_finish(const MapView &m, int mode, const MeshOut &out, const MeshScan &scan,
                              MeshReport *report, int schedule, MeshGrid grid, hipStream_t s)
{
    if (grid.emit < 1 || grid.count < grid.emit || grid.count > kMaxMeshGrid || grid.count % grid.emit ||
        grid.count / grid.emit > kMaxRecParts)
        return hipErrorInvalidValue;
    if (schedule == 0)
        hipLaunchKernelGGL(k_mesh_emit<0>, dim3(grid.emit), dim3(kThreads), 0, s, m, mode, scan, out, grid.count, report);
    else
        hipLaunchKernelGGL(k_mesh_emit<1>, dim3(grid.emit), dim3(kThreads), 0, s, m, mode, scan, out, grid.count, report);
    return hipGetLastError();
}

}  // namespace mc
