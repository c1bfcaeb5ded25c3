// Map-quality metrics of a reconstructed mesh against a ground-truth point cloud (Sec. V-C:
// the reconstruction error of Eq. 7, the Chamfer-L1 distance of Eq. 8, the reconstruction
// completeness, and the semantic scores mIoU and accuracy).
//
// Every distance the metrics use is capped at 2 nu, so each nearest-neighbour query only
// has to look 2 nu around its point: the reference cloud is bucketed in a uniform grid of
// cells slightly larger than the cap (an open-addressing hash of occupied cells, counts, an
// exclusive scan, and points scattered into per-cell runs as float4 with the point index in
// w), and a query scans the 27 cells around it.  Squared distances are fp64 sums of fp64
// differences of the fp32 coordinates, the nearest point the smallest (distance, index) pair.
// Sums are reduced in a fixed order (per-workgroup trees, then one workgroup), so results are
// bitwise reproducible.
#include "internal.h"

namespace mc {

constexpr int kQThreads = 256;
constexpr unsigned long long kNoCell = ~0ull;
constexpr int kCellBias = 1 << 20;  // cell coordinates are clamped to [-2^20, 2^20 - 1]

__device__ __forceinline__ int cell_coord(float x, double inv_h)
{
    double c = floor((double)x * inv_h);
    c = c < -(double)kCellBias ? -(double)kCellBias : (c > (double)(kCellBias - 1) ? (double)(kCellBias - 1) : c);
    return (int)c;
}

__device__ __forceinline__ unsigned long long cell_key(int cx, int cy, int cz)
{
    return ((unsigned long long)(cx + kCellBias) << 42) | ((unsigned long long)(cy + kCellBias) << 21) |
           (unsigned long long)(cz + kCellBias);
}

__global__ __launch_bounds__(kQThreads) void k_grid_insert(CellGrid g, const float *__restrict__ p, long long n)
{
    const long long i = blockIdx.x * (long long)kQThreads + threadIdx.x;
    if (i >= n) return;
    const float x = p[3 * i], y = p[3 * i + 1], z = p[3 * i + 2];
    const unsigned long long k = cell_key(cell_coord(x, g.inv_h), cell_coord(y, g.inv_h), cell_coord(z, g.inv_h));
    uint32_t s = hash_slot(k, g.mask);
    for (uint32_t probe = 0; probe <= g.mask; ++probe) {
        const unsigned long long prev = atomicCAS(&g.key[s], kNoCell, k);
        if (prev == kNoCell || prev == k) {
            atomicAdd(&g.count[s], 1u);
            g.slot_of[i] = s;
            return;
        }
        s = (s + 1) & g.mask;
    }
}

// Exclusive scan of the cell counts into offsets: per-workgroup scans, then the
// workgroup totals (one workgroup), then the totals added back.
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t *tmp, uint32_t *total)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t incl = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t y = __shfl_up(incl, off, 64);
        if (lane >= off) incl += y;
    }
    if (lane == 63) tmp[wave] = incl;
    __syncthreads();
    uint32_t before = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < kQThreads / 64; ++w) {
        before += w < wave ? tmp[w] : 0u;
        tot += tmp[w];
    }
    __syncthreads();
    *total = tot;
    return before + incl - v;
}

__global__ __launch_bounds__(kQThreads) void k_scan_blocks(const uint32_t *__restrict__ in, uint32_t *out,
                                                           uint32_t *block_sums, long long n)
{
    __shared__ uint32_t tmp[kQThreads / 64];
    const long long i = blockIdx.x * (long long)kQThreads + threadIdx.x;
    const uint32_t v = i < n ? in[i] : 0u;
    uint32_t tot;
    const uint32_t ex = block_exclusive_scan(v, tmp, &tot);
    if (i < n) out[i] = ex;
    if (threadIdx.x == 0) block_sums[blockIdx.x] = tot;
}

// One workgroup: exclusive scan of nb block sums in place (sequential chunks of kQThreads).
__global__ __launch_bounds__(kQThreads) void k_scan_top(uint32_t *block_sums, int nb)
{
    __shared__ uint32_t tmp[kQThreads / 64];
    uint32_t carry = 0;
    for (int base = 0; base < nb; base += kQThreads) {
        const int i = base + threadIdx.x;
        const uint32_t v = i < nb ? block_sums[i] : 0u;
        uint32_t tot;
        const uint32_t ex = block_exclusive_scan(v, tmp, &tot);
        if (i < nb) block_sums[i] = carry + ex;
        carry += tot;
    }
}

__global__ __launch_bounds__(kQThreads) void k_scan_add(uint32_t *out, const uint32_t *__restrict__ block_sums,
                                                        long long n)
{
    const long long i = blockIdx.x * (long long)kQThreads + threadIdx.x;
    if (i < n) out[i] += block_sums[blockIdx.x];
}

__global__ __launch_bounds__(kQThreads) void k_grid_fill(CellGrid g, const float *__restrict__ p, long long n)
{
    const long long i = blockIdx.x * (long long)kQThreads + threadIdx.x;
    if (i >= n) return;
    const uint32_t s = g.slot_of[i];
    const uint32_t at = g.offset[s] + atomicAdd(&g.cursor[s], 1u);
    g.pts[at] = make_float4(p[3 * i], p[3 * i + 1], p[3 * i + 2], __int_as_float((int)i));
}

// Nearest point of the grid's cloud within the 27 cells around each query point: capped
// distance min(cap, d) (fp64) and, if nn is not null, the point's index (-1 when none lies
// within the cap).
__global__ __launch_bounds__(kQThreads) void k_grid_query(CellGrid g, const float *__restrict__ q, long long n,
                                                          double cap, double *dist, long long *nn)
{
    const long long i = blockIdx.x * (long long)kQThreads + threadIdx.x;
    if (i >= n) return;
    const float x = q[3 * i], y = q[3 * i + 1], z = q[3 * i + 2];
    const int cx = cell_coord(x, g.inv_h), cy = cell_coord(y, g.inv_h), cz = cell_coord(z, g.inv_h);
    double best = INFINITY;
    int best_i = -1;
    for (int dz = -1; dz <= 1; ++dz)
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
                const int ax = cx + dx, ay = cy + dy, az = cz + dz;
                if (ax < -kCellBias || ax >= kCellBias || ay < -kCellBias || ay >= kCellBias || az < -kCellBias ||
                    az >= kCellBias)
                    continue;
                const unsigned long long k = cell_key(ax, ay, az);
                uint32_t s = hash_slot(k, g.mask);
                int found = -1;
                for (uint32_t probe = 0; probe <= g.mask; ++probe) {
                    const unsigned long long hk = g.key[s];
                    if (hk == k) {
                        found = (int)s;
                        break;
                    }
                    if (hk == kNoCell) break;
                    s = (s + 1) & g.mask;
                }
                if (found < 0) continue;
                const uint32_t o = g.offset[found], c = g.count[found];
                for (uint32_t j = 0; j < c; ++j) {
                    const float4 r = g.pts[o + j];
                    const double ex = (double)r.x - (double)x, ey = (double)r.y - (double)y,
                                 ez = (double)r.z - (double)z;
                    const double d2 = (ex * ex + ey * ey) + ez * ez;
                    const int idx = __float_as_int(r.w);
                    if (d2 < best || (d2 == best && idx < best_i)) {
                        best = d2;
                        best_i = idx;
                    }
                }
            }
    const double d = sqrt(best);
    const bool within = best_i >= 0 && d <= cap;
    dist[i] = within ? d : cap;
    if (nn) nn[i] = within ? best_i : -1;
}

// Per-workgroup partial sums over the mesh side (sum of d^2 and of d) and the ground-truth
// side (sum of d, covered points), in a fixed tree order; confusion counts
// [pred (L = none)][gt] of the covered ground-truth points, gathered in LDS per workgroup
// when (L + 1) L <= kConfLds (one global atomic per non-zero bin and workgroup), else
// straight to global memory.
constexpr int kQParts = 4;
constexpr int kConfLds = 4096;
__global__ __launch_bounds__(kQThreads) void k_quality_partials(const double *__restrict__ dM, long long nM,
                                                                const double *__restrict__ dG,
                                                                const long long *__restrict__ nnG, long long nG,
                                                                const uint8_t *__restrict__ labM,
                                                                const uint8_t *__restrict__ labG, int L,
                                                                double cap, double *partial,
                                                                unsigned long long *conf)
{
    __shared__ double red[kQParts][kQThreads];
    __shared__ uint32_t s_conf[kConfLds];
    const int nbins = (L + 1) * L;
    const bool in_lds = nbins <= kConfLds;
    if (in_lds)
        for (int b = threadIdx.x; b < nbins; b += kQThreads) s_conf[b] = 0u;
    __syncthreads();
    double acc[kQParts] = {0.0, 0.0, 0.0, 0.0};
    const long long stride = (long long)gridDim.x * kQThreads;
    for (long long i = blockIdx.x * (long long)kQThreads + threadIdx.x; i < nM; i += stride) {
        const double d = dM[i];
        acc[0] += d * d;
        acc[1] += d;
    }
    for (long long i = blockIdx.x * (long long)kQThreads + threadIdx.x; i < nG; i += stride) {
        const double d = dG[i];
        acc[2] += d;
        const long long j = nnG[i];
        if (j >= 0) {
            acc[3] += 1.0;
            const int gt = labG[i];
            if (gt < L) {
                const int pr = labM[j] < L ? labM[j] : L;
                if (in_lds) atomicAdd(&s_conf[pr * L + gt], 1u);
                else atomicAdd(&conf[(size_t)pr * L + gt], 1ull);
            }
        }
    }
    __syncthreads();
    if (in_lds)
        for (int b = threadIdx.x; b < nbins; b += kQThreads)
            if (s_conf[b]) atomicAdd(&conf[b], (unsigned long long)s_conf[b]);
#pragma unroll
    for (int k = 0; k < kQParts; ++k) red[k][threadIdx.x] = acc[k];
    __syncthreads();
    for (int s = kQThreads / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s)
#pragma unroll
            for (int k = 0; k < kQParts; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x < kQParts) partial[(size_t)blockIdx.x * kQParts + threadIdx.x] = red[threadIdx.x][0];
}

// One workgroup: the partials in a fixed order, then RE, CD, RC, mIoU and accuracy.
__global__ __launch_bounds__(kQThreads) void k_quality_final(const double *__restrict__ partial, int nparts,
                                                             const unsigned long long *__restrict__ conf, int L,
                                                             long long nM, long long nG, double *out)
{
    __shared__ double red[kQParts][kQThreads];
    double acc[kQParts] = {0.0, 0.0, 0.0, 0.0};
    for (int b = threadIdx.x; b < nparts; b += kQThreads)
#pragma unroll
        for (int k = 0; k < kQParts; ++k) acc[k] += partial[(size_t)b * kQParts + k];
#pragma unroll
    for (int k = 0; k < kQParts; ++k) red[k][threadIdx.x] = acc[k];
    __syncthreads();
    for (int s = kQThreads / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s)
#pragma unroll
            for (int k = 0; k < kQParts; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x != 0) return;
    const double sM2 = red[0][0], sM = red[1][0], sG = red[2][0], covered = red[3][0];
    const double re = nM ? sqrt(sM2 / (double)nM) : 0.0;
    const double cd = (nM ? 0.5 * (sM / (double)nM) : 0.0) + (nG ? 0.5 * (sG / (double)nG) : 0.0);
    const double rc = nG ? covered / (double)nG : 0.0;
    // per class: TP on the diagonal, FP the rest of its prediction row, FN the rest of its
    // ground-truth column (the "none" row included)
    double iou_sum = 0.0;
    long long n_occ = 0, tp_sum = 0, n_eval = 0;
    for (int c = 0; c < L; ++c) {
        long long tp = (long long)conf[(size_t)c * L + c], row = 0, col = 0;
        for (int j = 0; j < L; ++j) row += (long long)conf[(size_t)c * L + j];
        for (int j = 0; j <= L; ++j) col += (long long)conf[(size_t)j * L + c];
        const long long fp = row - tp, fn = col - tp;
        n_eval += col;
        tp_sum += tp;
        if (tp + fp + fn > 0) {
            iou_sum += (double)tp / (double)(tp + fp + fn);
            n_occ++;
        }
    }
    out[0] = re;
    out[1] = cd;
    out[2] = rc;
    out[3] = n_occ ? iou_sum / (double)n_occ : 0.0;
    out[4] = n_eval ? (double)tp_sum / (double)n_eval : 0.0;
    out[5] = (double)n_eval;
}

// ---------------------------------------------------------------------------------
// launch wrappers
// ---------------------------------------------------------------------------------

static int qgrid(long long n) { return (int)((n + kQThreads - 1) / kQThreads); }

hipError_t launch_grid_build(CellGrid &g, const float *p, long long n, uint32_t *scan_tmp, hipStream_t s)
{
    const long long slots = (long long)g.mask + 1;
    if (n > 0) hipLaunchKernelGGL(k_grid_insert, dim3(qgrid(n)), dim3(kQThreads), 0, s, g, p, n);
    const int nb = qgrid(slots);
    hipLaunchKernelGGL(k_scan_blocks, dim3(nb), dim3(kQThreads), 0, s, g.count, g.offset, scan_tmp, slots);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kQThreads), 0, s, scan_tmp, nb);
    hipLaunchKernelGGL(k_scan_add, dim3(nb), dim3(kQThreads), 0, s, g.offset, scan_tmp, slots);
    if (n > 0) hipLaunchKernelGGL(k_grid_fill, dim3(qgrid(n)), dim3(kQThreads), 0, s, g, p, n);
    return hipGetLastError();
}

hipError_t launch_grid_query(const CellGrid &g, const float *q, long long n, double cap, double *dist, long long *nn,
                             hipStream_t s)
{
    if (n > 0) hipLaunchKernelGGL(k_grid_query, dim3(qgrid(n)), dim3(kQThreads), 0, s, g, q, n, cap, dist, nn);
    return hipGetLastError();
}

hipError_t launch_quality(const double *dM, long long nM, const double *dG, const long long *nnG, long long nG,
                          const uint8_t *labM, const uint8_t *labG, int L, double cap, double *partial, int nparts,
                          unsigned long long *conf, double *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_quality_partials, dim3(nparts), dim3(kQThreads), 0, s, dM, nM, dG, nnG, nG, labM, labG, L,
                       cap, partial, conf);
    hipLaunchKernelGGL(k_quality_final, dim3(1), dim3(kQThreads), 0, s, partial, nparts, conf, L, nM, nG, out);
    return hipGetLastError();
}

}  // namespace mc
