// LiDAR integration kernels: block allocation (exact band-segment walk + hash), the
// projective TSDF update of Eq. 5, dirty-set marking, and camera label fusion (Eq. 6).
//
// Every value that is stored or decides which block, pixel or voxel is touched is
// computed in fp32 with a fixed evaluation order (the library is built with
// -ffp-contract=off); point-vs-pixel-boundary decisions are exact signs of fp64
// products of fp32 operands; the segment walk is exact integer arithmetic.
#include "internal.h"

namespace mc {

constexpr int kThreads = 256;
constexpr int kLdsKeys = 2048;  // per-workgroup de-duplication table (16 KiB)

// ---------------------------------------------------------------------------------
// pool initialisation and small helpers
// ---------------------------------------------------------------------------------

__global__ void k_fill_u64(unsigned long long *p, size_t n, unsigned long long v)
{
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = v;
}

hipError_t launch_fill_u64(unsigned long long *p, size_t n, unsigned long long v, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    size_t blocks = (n + kThreads - 1) / kThreads;
    int grid = (int)(blocks < 65536 ? blocks : 65536);
    hipLaunchKernelGGL(k_fill_u64, dim3(grid), dim3(kThreads), 0, s, p, n, v);
    return hipGetLastError();
}

// Fused labels start at 255 (unknown); D, W, counts and flags start at zero, which the
// caller clears with a device memset at create.
__global__ void k_init_fused(uint8_t *fused, size_t n)
{
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        reinterpret_cast<uint32_t *>(fused)[i] = 0xFFFFFFFFu;
}

hipError_t launch_init_pool(const MapView &m, hipStream_t s)
{
    size_t words = (size_t)m.max_blocks * kBlockVoxels / 4;
    size_t blocks = (words + kThreads - 1) / kThreads;
    int grid = (int)(blocks < 65536 ? blocks : 65536);
    hipLaunchKernelGGL(k_init_fused, dim3(grid), dim3(kThreads), 0, s, m.fused, words);
    return hipGetLastError();
}

__global__ void k_frame_begin(Counters *c)
{
    c->n_touched = 0;
    c->n_new = 0;
    c->frame_ok = 0;
    c->updates = 0;
    c->votes = 0;
    c->overflow = 0;
}

hipError_t launch_frame_begin(const MapView &m, hipStream_t s)
{
    hipLaunchKernelGGL(k_frame_begin, dim3(1), dim3(1), 0, s, m.ctr);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------------
// exact predicates and the nearest pixel
// ---------------------------------------------------------------------------------

// sign of ax*qy - ay*qx: the fp64 products of fp32 operands are exact, so the sign of the
// correctly rounded difference is exact
__device__ __forceinline__ double cross64(float ax, float ay, float qx, float qy)
{
    return (double)ax * (double)qy - (double)ay * (double)qx;
}

// Column c holds points strictly counter-clockwise of boundary c+1 and clockwise of, or
// on, boundary c (boundary c lies between columns c-1 and c; ties go to the higher index).
__device__ __forceinline__ bool col_holds(const LidarLUT &L, int c, float px, float py)
{
    int c1 = (c + 1 == L.cols) ? 0 : c + 1;
    return cross64(L.bcx[c1], L.bcy[c1], px, py) > 0.0 && cross64(L.bcx[c], L.bcy[c], px, py) <= 0.0;
}

// nearest pixel of a sensor-frame point, or false
__device__ __forceinline__ bool nearest_pixel(const LidarLUT &L, float px, float py, float pz, int &row,
                                              int &col)
{
    if (px == 0.0f && py == 0.0f) return false;
    const float kPi = 3.14159265358979f;
    float a = (kPi - atan2f(py, px)) * L.cols_over_2pi;
    int g = (int)floorf(a + 0.5f);
    g %= L.cols;
    if (g < 0) g += L.cols;
    int c = -1;
    if (col_holds(L, g, px, py)) c = g;
    else {
        int gm = g == 0 ? L.cols - 1 : g - 1, gp = g + 1 == L.cols ? 0 : g + 1;
        if (col_holds(L, gm, px, py)) c = gm;
        else if (col_holds(L, gp, px, py)) c = gp;
        else {
            for (int k = 0; k < L.cols; ++k)
                if (col_holds(L, k, px, py)) { c = k; break; }
            if (c < 0) return false;
        }
    }
    float rho = sqrtf(px * px + py * py);
    // inside the vertical field of view: on or below boundary 0, strictly above boundary R
    if (cross64(L.brc[0], L.brs[0], rho, pz) > 0.0) return false;
    if (cross64(L.brc[L.rows], L.brs[L.rows], rho, pz) <= 0.0) return false;
    // largest k in [0, rows-1] with the point on or below boundary k
    int lo = 0, hi = L.rows - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (cross64(L.brc[mid], L.brs[mid], rho, pz) <= 0.0) lo = mid;
        else hi = mid - 1;
    }
    row = lo;
    col = c;
    return true;
}

__device__ __forceinline__ bool valid_return(float r, float r_max)
{
    return isfinite(r) && r > 0.0f && r <= r_max;
}

// ---------------------------------------------------------------------------------
// allocation: band segment -> blocks, frame set, touched list
// ---------------------------------------------------------------------------------

// Insert into the frame set; the first inserter appends the block to the touched list
// and looks it up in the map.
__device__ void frame_insert(const MapView &m, const FrameView &f, unsigned long long key)
{
    uint32_t i = hash_slot(key, f.fmask);
    for (uint32_t n = 0; n <= f.fmask; ++n) {
        unsigned long long cur = __atomic_load_n(&f.fkeys[i], __ATOMIC_RELAXED);
        if (cur == key) return;
        if (cur == kEmpty) {
            unsigned long long prev = atomicCAS(&f.fkeys[i], kEmpty, key);
            if (prev == kEmpty) {
                int idx = atomicAdd(&m.ctr->n_touched, 1);
                if (idx < f.tk_cap) {
                    f.tk_key[idx] = key;
                    f.tk_fslot[idx] = (int)i;
                    int s = hash_find(m, key);
                    f.tk_slot[idx] = s;
                    f.tk_rank[idx] = s < 0 ? atomicAdd(&m.ctr->n_new, 1) : -1;
                } else {
                    atomicExch(&m.ctr->overflow, 1);
                }
                return;
            }
            if (prev == key) return;
        }
        i = (i + 1) & f.fmask;
    }
    atomicExch(&m.ctr->overflow, 1);
}

__device__ __forceinline__ void lds_or_global_insert(unsigned long long *lk, const MapView &m,
                                                     const FrameView &f, unsigned long long key)
{
    uint32_t i = hash_slot(key, kLdsKeys - 1);
    for (int n = 0; n < kLdsKeys; ++n) {
        unsigned long long cur = lk[i];
        if (cur == key) return;
        if (cur == kEmpty) {
            unsigned long long prev = atomicCAS(&lk[i], kEmpty, key);
            if (prev == kEmpty || prev == key) return;
        }
        i = (i + 1) & (kLdsKeys - 1);
    }
    frame_insert(m, f, key);  // table full: go straight to the frame set
}

// One thread per pixel.  The band segment of a valid return, in 2^-16-voxel fixed point
// (voxel v spans [v, v+1) after the half-voxel shift), is walked block by block: at each
// step the axis whose next block boundary comes first is advanced.  Moves in the
// positive direction happen at the crossing parameter (the boundary plane belongs to the
// next block); moves in the negative direction happen just after it.  Axes with equal
// parameter and direction class move together, so a segment through an edge or corner
// skips the side blocks exactly as the half-open cells require.
__global__ __launch_bounds__(kThreads) void k_alloc(MapView m, FrameView f, LidarLUT L, Pose T,
                                                   const float *__restrict__ range)
{
    __shared__ unsigned long long lk[kLdsKeys];
    for (int i = threadIdx.x; i < kLdsKeys; i += kThreads) lk[i] = kEmpty;
    __syncthreads();

    const int npix = L.rows * L.cols;
    const int pix = blockIdx.x * kThreads + threadIdx.x;
    if (pix < npix) {
        float r = range[pix];
        if (valid_return(r, L.r_max)) {
            const int k = pix / L.cols, c = pix - k * L.cols;
            const float dx = L.ce[k] * L.cp[c], dy = L.ce[k] * L.sp[c], dz = L.se[k];
            float s0 = r - m.tau;
            if (!(s0 > 0.0f)) s0 = 0.0f;
            const float s1 = r + m.tau;
            long long Q0[3], Q1[3], b[3], be[3], d[3];
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const float w = (T.m[4 * a] * dx + T.m[4 * a + 1] * dy) + T.m[4 * a + 2] * dz;
                const float o = T.m[4 * a + 3];
                const float p0 = o + s0 * w, p1 = o + s1 * w;
                const float q0 = p0 / m.nu + 0.5f, q1 = p1 / m.nu + 0.5f;
                Q0[a] = (long long)rintf(q0 * 65536.0f);
                Q1[a] = (long long)rintf(q1 * 65536.0f);
                b[a] = Q0[a] >> 19;   // arithmetic shift: floor division by one block
                be[a] = Q1[a] >> 19;
                d[a] = Q1[a] - Q0[a];
            }
            lds_or_global_insert(lk, m, f, pack_key((int)b[0], (int)b[1], (int)b[2]));
            for (int step = 0; step < 64; ++step) {
                if (b[0] == be[0] && b[1] == be[1] && b[2] == be[2]) break;
                long long bn = 0, bm = 1;
                int bcls = 2;
                long long n[3], mm[3];
                int cls[3];
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    cls[a] = 2;  // no event
                    if (b[a] == be[a]) continue;
                    if (d[a] > 0) {
                        n[a] = ((b[a] + 1) << 19) - Q0[a];
                        mm[a] = d[a];
                        cls[a] = 0;
                    } else {
                        n[a] = Q0[a] - (b[a] << 19);
                        mm[a] = -d[a];
                        cls[a] = 1;
                    }
                    bool earlier;
                    if (bcls == 2) earlier = true;
                    else {
                        long long lhs = n[a] * bm, rhs = bn * mm[a];
                        earlier = lhs < rhs || (lhs == rhs && cls[a] < bcls);
                    }
                    if (earlier) { bn = n[a]; bm = mm[a]; bcls = cls[a]; }
                }
#pragma unroll
                for (int a = 0; a < 3; ++a)
                    if (cls[a] == bcls && n[a] * bm == bn * mm[a]) b[a] += d[a] > 0 ? 1 : -1;
                lds_or_global_insert(lk, m, f, pack_key((int)b[0], (int)b[1], (int)b[2]));
            }
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kLdsKeys; i += kThreads) {
        unsigned long long key = lk[i];
        if (key != kEmpty) frame_insert(m, f, key);
    }
}

hipError_t launch_alloc(const MapView &m, const FrameView &f, const LidarLUT &lut, const Pose &T,
                        const float *range, hipStream_t s)
{
    int npix = lut.rows * lut.cols;
    int grid = (npix + kThreads - 1) / kThreads;
    hipLaunchKernelGGL(k_alloc, dim3(grid), dim3(kThreads), 0, s, m, f, lut, T, range);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------------
// TSDF integration (Eq. 5), one workgroup per touched block
// ---------------------------------------------------------------------------------

__device__ __forceinline__ void hash_insert(const MapView &m, unsigned long long key, int slot)
{
    uint32_t i = hash_slot(key, m.hmask);
    for (uint32_t n = 0; n <= m.hmask; ++n) {
        unsigned long long prev = atomicCAS(&m.hkeys[i], kEmpty, key);
        if (prev == kEmpty) {
            m.hvals[i] = slot;
            return;
        }
        i = (i + 1) & m.hmask;
    }
}

__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long v)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__global__ __launch_bounds__(kThreads) void k_tsdf(MapView m, FrameView f, LidarLUT L, Pose T,
                                                  const float *__restrict__ range)
{
    __shared__ int s_slot;
    __shared__ unsigned long long s_sum[kThreads / 64];
    Counters *c = m.ctr;
    const int n_touched = c->n_touched;
    const int n_new = c->n_new;
    const int used = c->pool_used;
    const bool ok = c->overflow == 0 && n_touched <= f.tk_cap && used + n_new <= m.max_blocks;
    if (!ok) {
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            c->frame_ok = 0;
            c->status = -2;  // MAP_ERR_CAPACITY, reported by the next synchronising call
        }
        return;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) c->frame_ok = 1;

    const float nu = m.nu, tau = m.tau, two_tau = m.tau + m.tau;
    unsigned long long my_updates = 0;
    for (int e = blockIdx.x; e < n_touched; e += gridDim.x) {
        const unsigned long long key = f.tk_key[e];
        if (threadIdx.x == 0) {
            int slot = f.tk_slot[e];
            if (slot < 0) {  // commit a new block: slot after the used ones, in rank order
                slot = used + f.tk_rank[e];
                hash_insert(m, key, slot);
                int3 bc = unpack_key(key);
                m.coords[slot] = make_int4(bc.x, bc.y, bc.z, 0);
                f.tk_slot[e] = slot;
            }
            s_slot = slot;
        }
        __syncthreads();
        const int slot = s_slot;
        const int3 bc = unpack_key(key);
        float2 *dwb = m.dw + (size_t)slot * kBlockVoxels;
#pragma unroll
        for (int it = 0; it < kBlockVoxels / kThreads; ++it) {
            const int li = it * kThreads + threadIdx.x;
            const int vx = 8 * bc.x + (li & 7), vy = 8 * bc.y + ((li >> 3) & 7), vz = 8 * bc.z + (li >> 6);
            const float x = (float)vx * nu, y = (float)vy * nu, z = (float)vz * nu;
            const float dx = x - T.m[3], dy = y - T.m[7], dz = z - T.m[11];
            const float px = (T.m[0] * dx + T.m[4] * dy) + T.m[8] * dz;
            const float py = (T.m[1] * dx + T.m[5] * dy) + T.m[9] * dz;
            const float pz = (T.m[2] * dx + T.m[6] * dy) + T.m[10] * dz;
            bool band = false;
            int row, col;
            if (!(px == 0.0f && py == 0.0f && pz == 0.0f) && nearest_pixel(L, px, py, pz, row, col)) {
                const float r = range[row * L.cols + col];
                if (valid_return(r, L.r_max)) {
                    const float dist = sqrtf((px * px + py * py) + pz * pz);
                    const float psi = r - dist;
                    if (!(psi < -tau)) {
                        float w = (psi + tau) / two_tau;
                        if (w > 1.0f) w = 1.0f;
                        if (w != 0.0f) {
                            const float gam = psi < tau ? psi : tau;
                            float2 v = dwb[li];
                            const float num = v.y * v.x + w * gam;
                            const float den = v.y + w;
                            v.x = num / den;
                            v.y = den;
                            dwb[li] = v;
                            band = fabsf(psi) <= tau;
                            my_updates++;
                        }
                    }
                }
            }
            const unsigned long long bits = __ballot(band);
            if ((threadIdx.x & 63) == 0) f.band[(size_t)e * 8 + (li >> 6)] = bits;
        }
        __syncthreads();
    }
    unsigned long long w = wave_sum_u64(my_updates);
    if ((threadIdx.x & 63) == 0) s_sum[threadIdx.x >> 6] = w;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long t = 0;
        for (int i = 0; i < kThreads / 64; ++i) t += s_sum[i];
        if (t) atomicAdd(&c->updates, t);
    }
}

hipError_t launch_tsdf(const MapView &m, const FrameView &f, const LidarLUT &lut, const Pose &T,
                       const float *range, int grid, hipStream_t s)
{
    hipLaunchKernelGGL(k_tsdf, dim3(grid), dim3(kThreads), 0, s, m, f, lut, T, range);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------------
// frame end: dirty set (touched blocks and their lower neighbours), frame-set clear
// ---------------------------------------------------------------------------------

__device__ __forceinline__ void mark_dirty(const MapView &m, int slot, uint32_t epoch)
{
    uint32_t old = atomicExch(&m.dirty_flag[slot], epoch);
    if (old != epoch) {
        int i = atomicAdd(&m.ctr->n_dirty, 1);
        m.dirty_list[i] = slot;
    }
}

__global__ __launch_bounds__(kThreads) void k_finish(MapView m, FrameView f)
{
    Counters *c = m.ctr;
    const int n = min(c->n_touched, f.tk_cap);
    const bool ok = c->frame_ok != 0;
    const uint32_t epoch = c->dirty_epoch;
    for (int e = blockIdx.x * kThreads + threadIdx.x; e < n; e += gridDim.x * kThreads) {
        f.fkeys[f.tk_fslot[e]] = kEmpty;
        if (!ok) continue;
        const int3 b = unpack_key(f.tk_key[e]);
        mark_dirty(m, f.tk_slot[e], epoch);
        for (int j = 1; j < 8; ++j) {
            int s = hash_find(m, pack_key(b.x - (j & 1), b.y - ((j >> 1) & 1), b.z - ((j >> 2) & 1)));
            if (s >= 0) mark_dirty(m, s, epoch);
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        if (ok) {
            c->pool_used += c->n_new;
            c->frames += 1;
            c->last_touched = n;
            c->last_new = c->n_new;
        } else {
            c->last_touched = 0;  // a rejected frame leaves nothing to label
            c->last_new = 0;
        }
    }
}

hipError_t launch_finish(const MapView &m, const FrameView &f, int grid, hipStream_t s)
{
    hipLaunchKernelGGL(k_finish, dim3(grid), dim3(kThreads), 0, s, m, f);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------------
// label fusion (Eq. 6 as vote counts), one workgroup per touched block
// ---------------------------------------------------------------------------------

__global__ __launch_bounds__(kThreads) void k_labels(MapView m, FrameView f, Camera cam, Pose T,
                                                    const uint8_t *__restrict__ labels)
{
    __shared__ unsigned long long s_sum[kThreads / 64];
    Counters *c = m.ctr;
    const int n = c->last_touched;
    const float nu = m.nu;
    const float fw = (float)cam.width, fh = (float)cam.height;
    const int L = m.n_classes;
    unsigned long long my_votes = 0;
    for (int e = blockIdx.x; e < n; e += gridDim.x) {
        const int slot = f.tk_slot[e];
        const int3 bc = unpack_key(f.tk_key[e]);
#pragma unroll
        for (int it = 0; it < kBlockVoxels / kThreads; ++it) {
            const int li = it * kThreads + threadIdx.x;
            const unsigned long long bits = f.band[(size_t)e * 8 + (li >> 6)];
            if (bits == 0) continue;  // wave-uniform: one word per wave
            if (!((bits >> (li & 63)) & 1ull)) continue;
            const size_t vi = (size_t)slot * kBlockVoxels + li;
            if (!(m.dw[vi].y > 0.0f)) continue;
            const int vx = 8 * bc.x + (li & 7), vy = 8 * bc.y + ((li >> 3) & 7), vz = 8 * bc.z + (li >> 6);
            const float x = (float)vx * nu, y = (float)vy * nu, z = (float)vz * nu;
            const float dx = x - T.m[3], dy = y - T.m[7], dz = z - T.m[11];
            const float px = (T.m[0] * dx + T.m[4] * dy) + T.m[8] * dz;
            const float py = (T.m[1] * dx + T.m[5] * dy) + T.m[9] * dz;
            const float pz = (T.m[2] * dx + T.m[6] * dy) + T.m[10] * dz;
            if (!(pz > 0.0f)) continue;
            const float u = cam.fx * (px / pz) + cam.cx;
            const float v = cam.fy * (py / pz) + cam.cy;
            if (!(u >= 0.0f && u < fw && v >= 0.0f && v < fh)) continue;
            const int iu = (int)u, iv = (int)v;
            const int l = labels[(size_t)iv * cam.width + iu];
            if (l >= L) continue;
            uint16_t *cnt = m.counts + (size_t)slot * L * kBlockVoxels + li;
            unsigned cl = cnt[(size_t)l * kBlockVoxels];
            if (cl < 65535u) cl++;
            cnt[(size_t)l * kBlockVoxels] = (uint16_t)cl;
            const int fl = m.fused[vi];
            const unsigned cf = fl == 255 ? 0u : cnt[(size_t)fl * kBlockVoxels];
            if (l != fl && (cl > cf || (cl == cf && l < fl))) m.fused[vi] = (uint8_t)l;
            my_votes++;
        }
    }
    unsigned long long w = wave_sum_u64(my_votes);
    if ((threadIdx.x & 63) == 0) s_sum[threadIdx.x >> 6] = w;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long t = 0;
        for (int i = 0; i < kThreads / 64; ++i) t += s_sum[i];
        if (t) atomicAdd(&c->votes, t);
    }
}

hipError_t launch_labels(const MapView &m, const FrameView &f, const Camera &cam, const Pose &T,
                         const uint8_t *labels, int grid, hipStream_t s)
{
    hipLaunchKernelGGL(k_labels, dim3(grid), dim3(kThreads), 0, s, m, f, cam, T, labels);
    return hipGetLastError();
}

}  // namespace mc
