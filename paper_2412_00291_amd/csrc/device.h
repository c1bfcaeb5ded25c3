// Device bodies shared by the per-map kernels and the batched (many maps per launch)
// kernels, so both run the same arithmetic for a map.
//
// Every value that is stored or decides which block, pixel or voxel is touched is
// computed in fp32 with a fixed evaluation order (the library is built with
// -ffp-contract=off); point-vs-pixel-boundary decisions are exact signs of fp64
// products of fp32 operands; the segment walk is exact integer arithmetic.
#pragma once
#include "internal.h"

namespace mc {

constexpr int kLdsKeys = 2048;                    // per-workgroup de-duplication table (16 KiB)
constexpr int kKeysPerThread = kLdsKeys / kThreads;
constexpr int kHalo = 9;
constexpr int kHaloVoxels = kHalo * kHalo * kHalo;
constexpr size_t kMaxLdsLut = 40 * 1024;  // boundary tables staged in LDS up to this size

// ---------------------------------------------------------------------------------
// reductions
// ---------------------------------------------------------------------------------

__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long v)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Workgroup exclusive prefix sum of one int per thread; returns the exclusive prefix and
// writes the total to *total (all threads).  `tmp` holds kThreads / 64 ints.
__device__ __forceinline__ int wg_scan(int v, int *tmp, int *total)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int incl = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int y = __shfl_up(incl, off, 64);
        if (lane >= off) incl += y;
    }
    if (lane == 63) tmp[wave] = incl;
    __syncthreads();
    int before = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < kThreads / 64; ++w) {
        const int t = tmp[w];
        before += w < wave ? t : 0;
        tot += t;
    }
    __syncthreads();
    *total = tot;
    return before + incl - v;
}

// ---------------------------------------------------------------------------------
// exact predicates and the nearest pixel
// ---------------------------------------------------------------------------------

// sign of ax*qy - ay*qx: the fp64 products of fp32 operands are exact, so one fused
// multiply-add rounds the exact difference once (the same value as rounding the
// difference of the two exact products) and its sign is exact
__device__ __forceinline__ double cross64(float ax, float ay, float qx, float qy)
{
    return __builtin_fma((double)ax, (double)qy, -((double)ay * (double)qx));
}

// Square root rounded to nearest (the value of sqrtf) of x >= 0.  The hardware root is
// within one ulp of the root, so the rounded root is it or a neighbour: a neighbour s' is
// taken when the residual x - s' s (one fused multiply-add) says the root lies beyond the
// pair's geometric mean.  For x in [2^-64, FLT_MAX] the residuals stay normal numbers and
// their signs are exact; other arguments take sqrtf.
__device__ __forceinline__ float sqrt_rn(float x)
{
    if (!(x >= 0x1p-64f && x <= 3.40282347e38f)) return sqrtf(x);
    const float s = __builtin_amdgcn_sqrtf(x);
    const float sm = __int_as_float(__float_as_int(s) - 1), sp = __int_as_float(__float_as_int(s) + 1);
    float r = fmaf(-sm, s, x) <= 0.0f ? sm : s;
    r = fmaf(-sp, s, x) > 0.0f ? sp : r;
    return r;
}

// Column c holds points strictly counter-clockwise of boundary c+1 and clockwise of, or
// on, boundary c (boundary c lies between columns c-1 and c; ties go to the higher index).
__device__ __forceinline__ bool col_holds(const LidarLUT &L, int c, float px, float py)
{
    const int c1 = (c + 1 == L.cols) ? 0 : c + 1;
    const float2 b1 = L.bc[c1], b0 = L.bc[c];
    return cross64(b1.x, b1.y, px, py) > 0.0 && cross64(b0.x, b0.y, px, py) <= 0.0;
}

// Approximate atan2(y, x) for initial guesses only (the exact predicates decide): an odd
// polynomial in min/max(|x|, |y|) fitted (least squares, Lawson-weighted toward minimax)
// to atan on [0, 1], maximum error 1.2e-5 rad, far below half a pixel of any scan.
// Needs (x, y) != (0, 0).
__device__ __forceinline__ float atan2_guess(float y, float x)
{
    const float ax = fabsf(x), ay = fabsf(y);
    const float t = fminf(ax, ay) * __builtin_amdgcn_rcpf(fmaxf(ax, ay));
    const float s = t * t;
    float p = fmaf(s, 0.020848948f, -0.0851640022f);
    p = fmaf(p, s, 0.180164277f);
    p = fmaf(p, s, -0.330305951f);
    p = fmaf(p, s, 0.9998664f);
    float r = p * t;
    if (ay > ax) r = 1.57079633f - r;
    if (x < 0.0f) r = 3.14159265f - r;
    return y < 0.0f ? -r : r;
}

// nearest pixel of a sensor-frame point, or false
__device__ __forceinline__ bool nearest_pixel(const LidarLUT &L, float px, float py, float pz, int &row,
                                              int &col)
{
    if (px == 0.0f && py == 0.0f) return false;
    const float kPi = 3.14159265358979f;
    const float a = (kPi - atan2_guess(py, px)) * L.cols_over_2pi;
    // a is in [0, cols] up to the guess's error, so one wrap and a clamp give a valid start
    // (the exact predicates decide the column; no integer division on this path)
    int g = (int)floorf(a + 0.5f);
    g = g >= L.cols ? g - L.cols : g;
    g = g < 0 ? 0 : (g >= L.cols ? L.cols - 1 : g);
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
    // The row is the largest k in [0, rows-1] with the point on or below boundary k (the
    // boundaries descend with k); the point is inside the vertical field of view when it
    // is on or below boundary 0 and strictly above boundary rows.  Start from the
    // elevation's guess and walk with the exact predicates: down while the point is on or
    // below boundary k+1 (reaching boundary rows: outside), or up until it is on or below
    // boundary k (passing boundary 0: outside).  The walk's end implies the field-of-view
    // test, so the common case takes two predicates.
    const float rho = sqrt_rn(px * px + py * py);
    const int R = L.rows;
    int k = (int)floorf((L.el_top - atan2_guess(pz, rho)) * L.rows_over_fov);
    k = k < 0 ? 0 : (k > R - 1 ? R - 1 : k);
    float2 b = L.br[k];
    if (cross64(b.x, b.y, rho, pz) <= 0.0) {
        for (;;) {
            b = L.br[k + 1];
            if (cross64(b.x, b.y, rho, pz) > 0.0) break;
            if (k + 1 == R) return false;
            ++k;
        }
    } else {
        for (;;) {
            if (k == 0) return false;
            --k;
            b = L.br[k];
            if (cross64(b.x, b.y, rho, pz) <= 0.0) break;
        }
    }
    row = k;
    col = c;
    return true;
}

// Copy the boundary tables (column boundaries, then row boundaries) into the workgroup's
// LDS and point L at the copy; every thread calls it.  Every load of a chunk is in flight
// at once (2560 pairs per chunk: one chunk for 2048 columns).
__device__ __forceinline__ void stage_lut(LidarLUT &L, float2 *s_lut)
{
    constexpr int kPer = 10;
    const int nc = L.cols, n = L.cols + L.rows + 1;
    for (int i0 = 0; i0 < n; i0 += kPer * kThreads) {
        float2 v[kPer];
#pragma unroll
        for (int k = 0; k < kPer; ++k) {
            const int i = i0 + k * kThreads + (int)threadIdx.x;
            const float2 *src = i < nc ? L.bc + i : L.br + (i - nc);  // one load per element
            v[k] = make_float2(0.0f, 0.0f);
            if (i < n) v[k] = *src;
        }
#pragma unroll
        for (int k = 0; k < kPer; ++k) {
            const int i = i0 + k * kThreads + (int)threadIdx.x;
            if (i < n) s_lut[i] = v[k];
        }
    }
    L.bc = s_lut;
    L.br = s_lut + nc;
    __syncthreads();
}

__device__ __forceinline__ bool valid_return(float r, float r_max)
{
    return isfinite(r) && r > 0.0f && r <= r_max;
}

// ---------------------------------------------------------------------------------
// allocation: band segment -> blocks, frame set, touched list
// ---------------------------------------------------------------------------------

// Claim a key in the frame set: 1 if this call inserted it (first in the frame), 0 if it
// was there, -1 if the set is full.  Writes the set slot to *slot.
__device__ __forceinline__ int frame_claim_from(const FrameView &f, unsigned long long key, uint32_t i, uint32_t n0,
                                                uint32_t *slot)
{
    for (uint32_t n = n0; n <= f.fmask; ++n) {
        const unsigned long long prev = atomicCAS(&f.fkeys[i], kEmpty, key);
        if (prev == kEmpty) {
            *slot = i;
            return 1;
        }
        if (prev == key) return 0;
        i = (i + 1) & f.fmask;
    }
    return -1;
}

__device__ __forceinline__ int frame_claim(const FrameView &f, unsigned long long key, uint32_t *slot)
{
    return frame_claim_from(f, key, hash_slot(key, f.fmask), 0, slot);
}

// Slot of a key in the block hash, probing from slot i (probe n0 of the sequence).
__device__ __forceinline__ int hash_find_from(const MapView &m, unsigned long long key, uint32_t i, uint32_t n0)
{
    for (uint32_t n = n0; n <= m.hmask; ++n) {
        const HashEntry h = hash_entry(&m.hash[i]);
        if (h.key == key) return h.val;
        if (h.key == kEmpty) return -1;
        i = (i + 1) & m.hmask;
    }
    return -1;
}

// Direct insert used only when a workgroup's LDS table overflows: one atomic per block.
__device__ __forceinline__ void frame_insert_direct(const MapView &m, const FrameView &f, unsigned long long key)
{
    uint32_t fs;
    const int c = frame_claim(f, key, &fs);
    if (c < 0) atomicExch(&m.ctr->overflow, 1);
    if (c <= 0) return;
    const int s = hash_find(m, key);
    const unsigned long long add = 1ull | (s < 0 ? (1ull << 32) : 0ull);
    const unsigned long long old = atomicAdd(&m.ctr->touched_new, add);
    const int idx = (int)(old & 0xFFFFFFFFull);
    if (idx >= f.tk_cap) {
        atomicExch(&m.ctr->overflow, 1);
        return;
    }
    f.tk_key[idx] = key;
    f.tk_fslot[idx] = (int)fs;
    f.tk_slot[idx] = s;
    f.tk_rank[idx] = s < 0 ? (int)(old >> 32) : -1;
}

__device__ __forceinline__ void lds_insert(unsigned long long *lk, const MapView &m, const FrameView &f,
                                           unsigned long long key)
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
    frame_insert_direct(m, f, key);  // table full: straight to the frame set
}

// Normal image and point filter of the non-projective distance (Sec. IV-C.2; the filter
// of Sec. V-C).  Pixel (k, c) back-projects to p = r d(k, c); its normal is the normalised
// cross product (p1 - p) x (p2 - p) of the differences to the pixel above, (k - 1, c), and
// the pixel to its left, (k, c - 1) with columns wrapping around the turn, turned to face
// the sensor.  The top row and pixels whose own or neighbouring return is invalid have
// none.  The return is kept when the angle between its ray and the normal is at most the
// incidence limit (cosine >= cos_inc).  Returns the normal rotated into the world frame in
// xyz and the kept range in w (all 0 when the return is not kept).  fp32, fixed order.
__device__ __forceinline__ float4 pixel_normal(const LidarLUT &L, const Pose &T, const float *__restrict__ range,
                                               int k, int c, float cos_inc)
{
    const int C = L.cols;
    const int ku = k > 0 ? k - 1 : 0, cl = c == 0 ? C - 1 : c - 1;  // clamped: row 0 reads itself
    const float r = range[k * C + c], r1 = range[ku * C + c], r2 = range[k * C + cl];
    const float cek = L.ce[k], sek = L.se[k], ceu = L.ce[ku], seu = L.se[ku];
    const float cpc = L.cp[c], spc = L.sp[c], cpl = L.cp[cl], spl = L.sp[cl];
    float4 out = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    if (k == 0 || !valid_return(r, L.r_max) || !valid_return(r1, L.r_max) || !valid_return(r2, L.r_max)) return out;
    const float dx = cek * cpc, dy = cek * spc, dz = sek;
    const float px = r * dx, py = r * dy, pz = r * dz;
    const float p1x = r1 * (ceu * cpc), p1y = r1 * (ceu * spc), p1z = r1 * seu;
    const float p2x = r2 * (cek * cpl), p2y = r2 * (cek * spl), p2z = r2 * sek;
    const float ax = p1x - px, ay = p1y - py, az = p1z - pz;
    const float bx = p2x - px, by = p2y - py, bz = p2z - pz;
    float nx = ay * bz - az * by, ny = az * bx - ax * bz, nz = ax * by - ay * bx;
    const float l2 = (nx * nx + ny * ny) + nz * nz;
    if (!(l2 > 0.0f) || !isfinite(l2)) return out;
    const float l = sqrt_rn(l2);
    nx = nx / l;
    ny = ny / l;
    nz = nz / l;
    float s = (nx * dx + ny * dy) + nz * dz;  // cosine between the normal and the ray
    if (s > 0.0f) {
        nx = -nx;
        ny = -ny;
        nz = -nz;
        s = -s;
    }
    if (!(-s >= cos_inc)) return out;
    out.x = (T.m[0] * nx + T.m[1] * ny) + T.m[2] * nz;
    out.y = (T.m[4] * nx + T.m[5] * ny) + T.m[6] * nz;
    out.z = (T.m[8] * nx + T.m[9] * ny) + T.m[10] * nz;
    out.w = r;
    return out;
}

// The band segment of one pixel's valid return, in 2^-16-voxel fixed point (voxel v
// spans [v, v+1) after the half-voxel shift), walked block by block: at each step the
// axis whose next block boundary comes first advances.  Moves in the positive direction
// happen at the crossing parameter (the boundary plane belongs to the next block); moves
// in the negative direction happen just after it.  Axes with equal parameter and
// direction class move together, so a segment through an edge or corner skips the side
// blocks exactly as the half-open cells require.  With the non-projective distance (kNP)
// the pixel's normal and point filter come first (stored in the frame's normal image),
// and the kept return is the one walked.
template <bool kNP = false, bool kCopy = false>
__device__ __forceinline__ void alloc_pixel(unsigned long long *lk, const MapView &m, const FrameView &f,
                                            const LidarLUT &L, const Pose &T, const float *__restrict__ range,
                                            int pix, float cos_inc = 0.0f)
{
    const int k = pix / L.cols, c = pix - k * L.cols;
    float r;
    if (kNP) {
        const float4 nr = pixel_normal(L, T, range, k, c, cos_inc);
        f.nimg[pix] = nr;
        r = nr.w;
    } else {
        r = range[pix];
        if (kCopy) f.rcopy[pix] = r;  // the frame's own copy, read by the TSDF launch
    }
    const float ce = L.ce[k], se = L.se[k], cp = L.cp[c], sp = L.sp[c];
    // the table reads wait here with the return (else the compiler moves them past the
    // validity test: a second round trip)
    asm volatile("" ::"v"(r), "v"(ce), "v"(se), "v"(cp), "v"(sp));
    if (!valid_return(r, L.r_max)) return;
    const float dx = ce * cp, dy = ce * sp, dz = se;
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
    lds_insert(lk, m, f, pack_key((int)b[0], (int)b[1], (int)b[2]));
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
        lds_insert(lk, m, f, pack_key((int)b[0], (int)b[1], (int)b[2]));
    }
}

// Claim the workgroup's de-duplicated blocks in the frame set; the first claimant of
// each block in the frame appends it to the touched list (with its map slot, or its rank
// among the frame's new blocks), with one list reservation per workgroup.  The LDS table
// is compacted first so that the claims (a dependent chain of global operations each)
// spread over all threads instead of one chain per table slot.
__device__ __forceinline__ void alloc_flush(unsigned long long *lk, int *s_tmp, unsigned long long *s_base,
                                            const MapView &m, const FrameView &f)
{
    unsigned long long key[kKeysPerThread];
    int n_mine = 0;
#pragma unroll
    for (int j = 0; j < kKeysPerThread; ++j) {
        key[j] = lk[threadIdx.x + j * kThreads];
        n_mine += key[j] != kEmpty;
    }
    int n_keys;
    int o = wg_scan(n_mine, s_tmp, &n_keys);  // its barriers also order the reads above
#pragma unroll
    for (int j = 0; j < kKeysPerThread; ++j)
        if (key[j] != kEmpty) lk[o++] = key[j];
    __syncthreads();
    uint32_t fslot[kKeysPerThread];
    int mslot[kKeysPerThread];
    int n_win = 0, n_new = 0;
#pragma unroll
    for (int j = 0; j < kKeysPerThread; ++j) {
        const int i = threadIdx.x + j * kThreads;
        mslot[j] = -2;  // not a winner
        if (i >= n_keys) continue;
        key[j] = lk[i];
        // the frame-set claim (a CAS at the key's first slot) and the block-hash probe are
        // issued together; either continues past its first slot only on a collision
        const uint32_t fi = hash_slot(key[j], f.fmask), hi = hash_slot(key[j], m.hmask);
        const unsigned long long prev = atomicCAS(&f.fkeys[fi], kEmpty, key[j]);
        const HashEntry h = hash_entry(&m.hash[hi]);
        asm volatile("" ::"v"(prev), "v"(h.key), "v"(h.val));  // both results wait here together
        int c;
        if (prev == kEmpty) {
            c = 1;
            fslot[j] = fi;
        } else {
            c = prev == key[j] ? 0 : frame_claim_from(f, key[j], (fi + 1) & f.fmask, 1, &fslot[j]);
        }
        if (c < 0) atomicExch(&m.ctr->overflow, 1);
        if (c <= 0) continue;
        mslot[j] = h.key == key[j] ? h.val : (h.key == kEmpty ? -1 : hash_find_from(m, key[j], (hi + 1) & m.hmask, 1));
        n_win++;
        n_new += mslot[j] < 0;
    }
    int tot_win, tot_new;
    const int off_win = wg_scan(n_win, s_tmp, &tot_win);
    const int off_new = wg_scan(n_new, s_tmp, &tot_new);
    if (threadIdx.x == 0)
        *s_base = tot_win ? atomicAdd(&m.ctr->touched_new, ((unsigned long long)tot_new << 32) | (unsigned)tot_win)
                          : 0ull;
    __syncthreads();
    int idx = (int)(*s_base & 0xFFFFFFFFull) + off_win;
    int rank = (int)(*s_base >> 32) + off_new;
#pragma unroll
    for (int j = 0; j < kKeysPerThread; ++j) {
        if (mslot[j] == -2) continue;
        if (idx < f.tk_cap) {
            f.tk_key[idx] = key[j];
            f.tk_fslot[idx] = (int)fslot[j];
            f.tk_slot[idx] = mslot[j];
            f.tk_rank[idx] = mslot[j] < 0 ? rank : -1;
        } else {
            atomicExch(&m.ctr->overflow, 1);
        }
        idx++;
        rank += mslot[j] < 0;
    }
}

// ---------------------------------------------------------------------------------
// TSDF integration (Eq. 5) with block commit and dirty marking
// ---------------------------------------------------------------------------------


template <class T>
__device__ __forceinline__ T coherent_load(T *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Wait until this thread's earlier memory operations (including atomics whose result is
// unused) have completed, so a following ticket atomic is performed after them.
__device__ __forceinline__ void wait_memory() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

// Frame state after allocation, read by a later launch (plain loads: the counters'
// last atomic updates were performed before that launch began).  Split in two so a
// launch can issue the loads before other start-up work and use them after it.
struct FrameRaw {
    unsigned long long tn;
    int32_t used, overflow;
    uint32_t epoch;
};

__device__ __forceinline__ FrameRaw frame_raw(const MapView &m)
{
    const Counters *c = m.ctr;
    FrameRaw r;
    r.tn = c->touched_new;
    r.used = c->pool_used;
    r.epoch = c->dirty_epoch;
    r.overflow = c->overflow;
    return r;
}

__device__ __forceinline__ FrameState frame_state_of(const FrameRaw &r, const MapView &m, const FrameView &f)
{
    FrameState s;
    const int n_touched = (int)(r.tn & 0xFFFFFFFFull);
    s.n_new = (int)(r.tn >> 32);
    s.used = r.used;
    s.epoch = r.epoch;
    s.ok = r.overflow == 0 && n_touched <= f.tk_cap && s.used + s.n_new <= m.max_blocks;
    s.n_list = n_touched < f.tk_cap ? n_touched : f.tk_cap;
    s.bits = s.used + s.n_new > m.bits_from;
    return s;
}

__device__ __forceinline__ FrameState frame_state(const MapView &m, const FrameView &f)
{
    return frame_state_of(frame_raw(m), m, f);
}

// The same, read in the launch whose atomics wrote the counters (device-coherent loads).
__device__ __forceinline__ FrameState frame_state_coherent(const MapView &m, const FrameView &f)
{
    Counters *c = m.ctr;
    const unsigned long long tn = coherent_load(&c->touched_new);
    FrameState s;
    const int n_touched = (int)(tn & 0xFFFFFFFFull);
    s.n_new = (int)(tn >> 32);
    s.used = coherent_load(&c->pool_used);
    s.epoch = coherent_load(&c->dirty_epoch);
    s.ok = coherent_load(&c->overflow) == 0 && n_touched <= f.tk_cap && s.used + s.n_new <= m.max_blocks;
    s.n_list = n_touched < f.tk_cap ? n_touched : f.tk_cap;
    s.bits = s.used + s.n_new > m.bits_from;
    return s;
}

// ---------------------------------------------------------------------------------
// spread counters and hierarchical tickets (no address takes more than ~64 atomics)
// ---------------------------------------------------------------------------------

__device__ __forceinline__ void spread_add(Spread &s, unsigned long long v)
{
    atomicAdd(&s.v[(blockIdx.x % kLeaves) * kLeafPad], v);
}

// Sum and clear a spread counter: called by one whole wavefront (lane l takes leaf l);
// every lane gets the sum.  Its caller is the counter's only user at that time.
__device__ __forceinline__ unsigned long long spread_take_wave(Spread &s)
{
    const int lane = threadIdx.x & 63;
    return wave_sum_u64(atomicExch(&s.v[lane * kLeafPad], 0ull));
}

// One thread per workgroup, after the workgroup's work: true in exactly one workgroup,
// the last to arrive, which also resets the ticket for the next launch.
__device__ __forceinline__ bool ticket_arrive(Ticket &t)
{
    const unsigned G = gridDim.x;
    const unsigned leaves = G < (unsigned)kLeaves ? G : (unsigned)kLeaves;
    const unsigned l = blockIdx.x % leaves;
    const unsigned long long expect = (G - l + leaves - 1) / leaves;  // workgroups of leaf l
    wait_memory();  // this workgroup's earlier memory operations complete first
    if (atomicAdd(&t.leaf[l * kLeafPad], 1ull) + 1ull != expect) return false;
    if (atomicAdd(&t.root[0], 1ull) + 1ull != leaves) return false;
    for (unsigned i = 0; i < leaves; ++i) atomicExch(&t.leaf[i * kLeafPad], 0ull);
    atomicExch(&t.root[0], 0ull);
    return true;
}

// The same ticket carrying a sum: each workgroup arrives with its count (below 2^40 in
// total), and the last one receives the launch's total in *total, so no counter has to be
// read back after the ticket.  Nothing the workgroups wrote is read in the launch, so a
// workgroup arrives without waiting for its stores.
__device__ __forceinline__ bool ticket_arrive_sum(Ticket &t, unsigned long long mine, unsigned long long *total)
{
    constexpr unsigned long long kOne = 1ull << 40, kMask = kOne - 1;
    const unsigned G = gridDim.x;
    const unsigned leaves = G < (unsigned)kLeaves ? G : (unsigned)kLeaves;
    const unsigned l = blockIdx.x % leaves;
    const unsigned long long expect = (G - l + leaves - 1) / leaves;  // workgroups of leaf l
    const unsigned long long o = atomicAdd(&t.leaf[l * kLeafPad], kOne | mine);
    if ((o >> 40) + 1ull != expect) return false;
    const unsigned long long leaf_sum = (o & kMask) + mine;
    const unsigned long long r = atomicAdd(&t.root[0], kOne | leaf_sum);
    if ((r >> 40) + 1ull != leaves) return false;
    *total = (r & kMask) + leaf_sum;
    for (unsigned i = 0; i < leaves; ++i) atomicExch(&t.leaf[i * kLeafPad], 0ull);
    atomicExch(&t.root[0], 0ull);
    return true;
}

// Insert a new block: claim the slot with a CAS on the key, then write the pool slot and
// the inserting call's number.  No other launch reads these before this one ends.
__device__ __forceinline__ void hash_insert_new(const MapView &m, unsigned long long key, int slot, uint32_t frame_id)
{
    uint32_t i = hash_slot(key, m.hmask);
    for (uint32_t n = 0; n <= m.hmask; ++n) {
        unsigned long long prev = atomicCAS(&m.hash[i].key, kEmpty, key);
        if (prev == kEmpty) {
            *reinterpret_cast<uint2 *>(&m.hash[i].val) = make_uint2((uint32_t)slot, frame_id);
            return;
        }
        i = (i + 1) & m.hmask;
    }
}

// Slot of a block that existed before this call, or -1 (absent, or inserted by this call:
// its slot may not be written yet, and it is in the touched list anyway).  A key seen
// before its tag is written reads the initial tag ~0 and is also taken as new.
__device__ __forceinline__ int hash_find_old(const MapView &m, unsigned long long key, uint32_t frame_id)
{
    uint32_t i = hash_slot(key, m.hmask);
    for (uint32_t n = 0; n <= m.hmask; ++n) {
        const HashEntry h = hash_entry(&m.hash[i]);
        if (h.key == key) return (h.frame == ~0u || h.frame == frame_id) ? -1 : h.val;
        if (h.key == kEmpty) return -1;
        i = (i + 1) & m.hmask;
    }
    return -1;
}

// Set a slot's bit in the dirty bitmap (layout: MapView::dbits).
__device__ __forceinline__ void mark_bit(const MapView &m, int slot)
{
    const uint32_t s = (uint32_t)slot, G = (uint32_t)m.bits_grid;
    const uint32_t j = s / G, w = s - j * G;
    atomicOr(&m.dbits[(size_t)w * (uint32_t)m.bits_wpw + (j >> 5)], 1u << (j & 31));
}

// Commit of touched entry e by one thread: clear its frame-set slot, and give a new block
// its pool slot (after the used ones, in rank order) and insert it.  Returns the slot.
__device__ __forceinline__ int commit_entry(const MapView &m, const FrameView &f, const FrameState &fs, int e,
                                            unsigned long long key, uint32_t frame_id)
{
    f.fkeys[f.tk_fslot[e]] = kEmpty;  // the frame set is empty again at frame end
    int slot = f.tk_slot[e];
    if (fs.ok && slot < 0) {
        slot = fs.used + f.tk_rank[e];
        const int3 bc = unpack_key(key);
        m.coords[slot] = make_int4(bc.x, bc.y, bc.z, (int)fs.epoch);  // a new block is dirty
        if (fs.bits) mark_bit(m, slot);
        hash_insert_new(m, key, slot, frame_id);
        f.tk_slot[e] = slot;
    }
    return slot;
}

// Mark a block dirty: its coordinates' fourth component holds the epoch; with bits, its
// bit in the dirty bitmap is set as well (several marks of one block set it again).
__device__ __forceinline__ void mark_dirty(const MapView &m, int slot, uint32_t epoch, bool bits)
{
    reinterpret_cast<int *>(&m.coords[slot])[3] = (int)epoch;
    if (bits) mark_bit(m, slot);
}

// Whether a block is dirty in epoch (one 4-byte read).
__device__ __forceinline__ bool is_dirty(const MapView &m, int slot, uint32_t epoch)
{
    return (uint32_t)reinterpret_cast<const int *>(&m.coords[slot])[3] == epoch;
}

// Dirty set: the block and its allocated lower neighbours b - e, e in {0,1}^3 (a
// neighbour that is new in this frame is itself in the touched list and marks itself).
// Returns the slot that neighbour j of the block at bc (slot `slot`) marks, or -1.
__device__ __forceinline__ int neighbour_slot(const MapView &m, int j, int3 bc, int slot, uint32_t frame_id)
{
    if (j == 0) return slot;
    return hash_find_old(m, pack_key(bc.x - (j & 1), bc.y - ((j >> 1) & 1), bc.z - ((j >> 2) & 1)), frame_id);
}

// Projective TSDF update (Eq. 5), split so that a lane's voxels overlap their memory
// reads: project a voxel to its nearest pixel (-1 if none, with the sensor-frame
// distance), then update from the pixel's return.

// Nearest pixel (row * cols + col, or -1) of voxel li of the block at bc, its distance,
// and its offset from the sensor in the map frame (dv).
__device__ __forceinline__ int tsdf_project(const MapView &m, const LidarLUT &L, const Pose &T, int3 bc, int li,
                                            float &dist, float3 &dv)
{
    const float nu = m.nu;
    const int vx = 8 * bc.x + (li & 7), vy = 8 * bc.y + ((li >> 3) & 7), vz = 8 * bc.z + (li >> 6);
    const float x = (float)vx * nu, y = (float)vy * nu, z = (float)vz * nu;
    const float dx = x - T.m[3], dy = y - T.m[7], dz = z - T.m[11];
    dv = make_float3(dx, dy, dz);
    const float px = (T.m[0] * dx + T.m[4] * dy) + T.m[8] * dz;
    const float py = (T.m[1] * dx + T.m[5] * dy) + T.m[9] * dz;
    const float pz = (T.m[2] * dx + T.m[6] * dy) + T.m[10] * dz;
    dist = 0.0f;
    int row, col;
    if (px == 0.0f && py == 0.0f && pz == 0.0f) return -1;
    if (!nearest_pixel(L, px, py, pz, row, col)) return -1;
    dist = sqrt_rn((px * px + py * py) + pz * pz);
    return row * L.cols + col;
}

// Update (D, W) in v from return r at distance dist; true if updated.  band: |psi| <= tau.
__device__ __forceinline__ bool tsdf_update(const MapView &m, const LidarLUT &L, float r, float dist, float2 &v,
                                            bool &band)
{
    const float tau = m.tau, two_tau = m.tau + m.tau;
    band = false;
    if (!valid_return(r, L.r_max)) return false;
    const float psi = r - dist;
    if (psi < -tau) return false;
    // w = min((psi + tau) / 2 tau, 1): a dividend of at least 2 tau gives a quotient of at
    // least 1 under any rounding, so the division is needed only below it
    const float a = psi + tau;
    float w = 1.0f;
    if (a < two_tau) w = a / two_tau;
    if (w == 0.0f) return false;
    const float gam = psi < tau ? psi : tau;
    const float num = v.y * v.x + w * gam;
    const float den = v.y + w;
    v.x = num / den;
    v.y = den;
    band = fabsf(psi) <= tau;
    return true;
}

// The non-projective update (Eq. 4 as read, Eq. 5): the weight is that of the projective
// psi, the truncated value is the distance d = -psi u.(e + n) / (1 + n.e) clamped to
// [-tau, tau], where u is the unit ray from the sensor to the voxel, n the normal of the
// voxel's pixel (nr.xyz, kept range in nr.w) and e the voxel's gradient g, or n where
// n.g <= 0 (no gradient yet, or one 90 degrees or more from the normal).  The gradient
// becomes the normalised weighted average of the normals, (W g + w n) / |W g + w n|.
// True if updated; band: |psi| <= tau.
__device__ __forceinline__ bool tsdf_update_np(const MapView &m, const LidarLUT &L, float4 nr, float dist, float3 dv,
                                               float2 &v, float3 &g, bool &band)
{
    const float tau = m.tau, two_tau = m.tau + m.tau;
    band = false;
    if (!valid_return(nr.w, L.r_max)) return false;
    const float psi = nr.w - dist;
    if (psi < -tau) return false;
    const float a = psi + tau;
    float w = 1.0f;
    if (a < two_tau) w = a / two_tau;
    if (w == 0.0f) return false;
    const float ng = (nr.x * g.x + nr.y * g.y) + nr.z * g.z;
    const bool use_g = ng > 0.0f;
    const float ex = use_g ? g.x : nr.x, ey = use_g ? g.y : nr.y, ez = use_g ? g.z : nr.z;
    const float ux = dv.x / dist, uy = dv.y / dist, uz = dv.z / dist;
    const float hx = ex + nr.x, hy = ey + nr.y, hz = ez + nr.z;
    const float uh = (ux * hx + uy * hy) + uz * hz;
    const float ne = (nr.x * ex + nr.y * ey) + nr.z * ez;
    const float d = -(psi * (uh / (1.0f + ne)));
    const float gam = d >= 0.0f ? (d < tau ? d : tau) : (d > -tau ? d : -tau);
    const float sx = v.y * g.x + w * nr.x, sy = v.y * g.y + w * nr.y, sz = v.y * g.z + w * nr.z;
    const float l2 = (sx * sx + sy * sy) + sz * sz;
    if (l2 > 0.0f && isfinite(l2)) {
        const float l = sqrt_rn(l2);
        g = make_float3(sx / l, sy / l, sz / l);
    }
    const float num = v.y * v.x + w * gam;
    const float den = v.y + w;
    v.x = num / den;
    v.y = den;
    band = fabsf(psi) <= tau;
    return true;
}

// The TSDF update of one touched block's voxels by one worker of kWidth lanes (rank is
// the lane's index in the worker); records the block's band bits.  Returns the updates.
// The lane's (D, W) loads are issued first, then its projections (LDS tables), then all
// of its range reads, so a block costs one memory round trip.  With the non-projective
// distance (kNP) the lane also loads its voxels' gradients with (D, W), and reads the
// normal image (normal and kept range in one 16-byte load) in place of the range image.
template <int kWidth, bool kNP = false>
__device__ __forceinline__ unsigned long long tsdf_block(const MapView &m, const FrameView &f, const LidarLUT &L,
                                                         const Pose &T, const float *__restrict__ range, int e,
                                                         unsigned long long key, int slot, int rank,
                                                         unsigned long long *s_band = nullptr)
{
    static_assert(kWidth % 64 == 0, "a wavefront covers whole z slices");
    constexpr int kV = kBlockVoxels / kWidth;
    const int3 bc = unpack_key(key);
    float2 *dwb = m.dw + (size_t)slot * kBlockVoxels;
    float *gb = kNP ? m.grad + (size_t)slot * 3 * kBlockVoxels : nullptr;
    float2 v[kV];
    float3 g[kV], dv[kV];
    float4 nr[kV];
    int pix[kV];
    float dist[kV], r[kV];
#pragma unroll
    for (int it = 0; it < kV; ++it) {
        const int li = it * kWidth + rank;
        v[it] = dwb[li];
        if (kNP) g[it] = make_float3(gb[li], gb[kBlockVoxels + li], gb[2 * kBlockVoxels + li]);
    }
#pragma unroll
    for (int it = 0; it < kV; ++it) pix[it] = tsdf_project(m, L, T, bc, it * kWidth + rank, dist[it], dv[it]);
#pragma unroll
    for (int it = 0; it < kV; ++it) {
        if (kNP) nr[it] = pix[it] >= 0 ? f.nimg[pix[it]] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        else r[it] = pix[it] >= 0 ? range[pix[it]] : 0.0f;
    }
    unsigned long long upd = 0;
#pragma unroll
    for (int it = 0; it < kV; ++it) {
        const int li = it * kWidth + rank;
        bool band = false;
        if (kNP) {
            if (pix[it] >= 0 && tsdf_update_np(m, L, nr[it], dist[it], dv[it], v[it], g[it], band)) {
                dwb[li] = v[it];
                gb[li] = g[it].x;
                gb[kBlockVoxels + li] = g[it].y;
                gb[2 * kBlockVoxels + li] = g[it].z;
                upd++;
            }
        } else if (pix[it] >= 0 && tsdf_update(m, L, r[it], dist[it], v[it], band)) {
            dwb[li] = v[it];
            upd++;
        }
        // the wavefront holds z slice li / 64: its band bits and its voxel masks
        const unsigned long long bits = __ballot(band);
        const unsigned long long sg = __ballot(v[it].x < 0.0f), ob = __ballot(v[it].y > 0.0f);
        if ((threadIdx.x & 63) == 0) {
            f.band[(size_t)e * 8 + (li >> 6)] = bits;
            m.vmask[(size_t)slot * 16 + (li >> 6)] = sg;
            m.vmask[(size_t)slot * 16 + 8 + (li >> 6)] = ob;
            if (s_band) s_band[li >> 6] = bits;  // the block's band words for fused label fusion
        }
    }
    return upd;
}

// Close the frame (one thread, after every worker of the TSDF phase has finished):
// commit the pool size, record the frame's counts, reset the per-frame counters.  The
// caller has taken the frame's update count from its spread counter and cleared the
// votes of the previous frame.
__device__ __forceinline__ void close_frame(const MapView &m, const FrameState &fs, unsigned long long updates)
{
    Counters *c = m.ctr;
    if (fs.ok) {
        c->pool_used = fs.used + fs.n_new;
        c->frames += 1;
        c->frame_ok = 1;
        c->last_touched = fs.n_list;
        c->last_new = fs.n_new;
        c->last_updates = updates;
        if (!fs.bits) c->bits_gap = 1;  // this frame's marks are not in the dirty bitmap
    } else {
        c->frame_ok = 0;
        c->status = -2;  // MAP_ERR_CAPACITY, reported by the next synchronising call
        c->last_touched = 0;  // a rejected frame leaves nothing to label
        c->last_new = 0;
        c->last_updates = 0;
    }
    c->touched_new = 0;
    c->overflow = 0;
}

// The last workgroup's part of closing a map's frame: wave 0 takes the update count (and,
// with clear_votes, clears the label votes of the previous frame; the per-map path clears
// them in its allocation launch instead, so a TSDF launch that also fuses labels keeps its
// own), then closes the frame.
__device__ __forceinline__ void close_frame_wave(const MapView &m, const FrameState &fs, bool clear_votes = true)
{
    const unsigned long long upd = spread_take_wave(m.sync->updates);
    if (clear_votes) (void)spread_take_wave(m.sync->votes);
    if ((threadIdx.x & 63) == 0) close_frame(m, fs, upd);
}

// ---------------------------------------------------------------------------------
// label fusion (Eq. 6 as vote counts): one band voxel, every camera of the set in order
// ---------------------------------------------------------------------------------

// Called only for band voxels of the last frame; a band voxel was updated by that frame,
// so its weight is positive and the W > 0 condition of the label update holds without a
// read of W.  The votes of the call's cameras apply in camera order; the lane first
// issues every camera's label read, then every count it needs (each camera's label and
// the fused label), applies the votes in registers (cameras voting the same label share
// the count), and writes each changed count once.
// Band voxels of a touched block, compacted: load the block's 8 band words and their
// prefix popcounts; band_select gives the voxel of the t-th set bit.
// Voxel index of the r-th set bit (r < popcount) of band word k.
__device__ __forceinline__ int band_bit(unsigned long long x, int k, int r)
{
    int pos = 0;
#pragma unroll
    for (int width = 32; width >= 1; width >>= 1) {
        const int c = __popcll(x & ((1ull << width) - 1ull));
        if (r >= c) {
            r -= c;
            x >>= width;
            pos += width;
        }
    }
    return 64 * k + pos;
}

struct BandWords {
    unsigned long long w[8];
    int pre[9];
};

__device__ __forceinline__ BandWords band_words(const FrameView &f, int e)
{
    BandWords b;
    b.pre[0] = 0;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        b.w[k] = f.band[(size_t)e * 8 + k];
        b.pre[k + 1] = b.pre[k] + __popcll(b.w[k]);
    }
    return b;
}

// The same from a block's eight band words in LDS.
__device__ __forceinline__ BandWords band_words_lds(const unsigned long long *w)
{
    BandWords b;
    b.pre[0] = 0;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        b.w[k] = w[k];
        b.pre[k + 1] = b.pre[k] + __popcll(b.w[k]);
    }
    return b;
}

__device__ __forceinline__ int band_select(const BandWords &b, int t)
{
    int k = 0;
#pragma unroll
    for (int j = 1; j < 8; ++j) k += b.pre[j] <= t ? 1 : 0;
    unsigned long long x = b.w[0];  // selects, not indexing: the arrays stay in registers
    int pk = 0;
#pragma unroll
    for (int j = 1; j < 8; ++j) {
        x = k == j ? b.w[j] : x;
        pk = k == j ? b.pre[j] : pk;
    }
    return band_bit(x, k, t - pk);
}

// A workgroup's band voxels over a group of up to kLabGroup touched entries, as one flat
// list: the entries' band words, slots and keys in LDS, each entry's word prefix, and the
// entries' voxel prefix, so the workgroup's threads take consecutive voxels of the whole
// group in one pass instead of one entry after another.
constexpr int kLabGroup = 8;
struct LabelGroup {
    unsigned long long w[kLabGroup][8];
    unsigned long long key[kLabGroup];
    int slot[kLabGroup];
    int pre[kLabGroup][9];
};

// Voxel t (< the group's total) of the group: entry j, voxel index li.
__device__ __forceinline__ void label_group_voxel(const LabelGroup &g, const int *epre, int t, int &j, int &li)
{
    j = 0;
#pragma unroll
    for (int i = 1; i < kLabGroup; ++i) j += epre[i] <= t ? 1 : 0;
    int base = 0;  // selects, not indexing: epre stays in registers
#pragma unroll
    for (int i = 1; i < kLabGroup; ++i) base = j == i ? epre[i] : base;
    const int local = t - base;
    int k = 0;
#pragma unroll
    for (int i = 1; i < 8; ++i) k += g.pre[j][i] <= local ? 1 : 0;
    li = band_bit(g.w[j][k], k, local - g.pre[j][k]);
}

constexpr int kCamChunk = 4;  // cameras whose votes one pass gathers (register budget)

__device__ __forceinline__ int label_voxel(const MapView &m, const CameraSet &cs, int slot, int3 bc, int li)
{
    const size_t vi = (size_t)slot * kBlockVoxels + li;
    const float nu = m.nu;
    const int L = m.n_classes;
    const int vx = 8 * bc.x + (li & 7), vy = 8 * bc.y + ((li >> 3) & 7), vz = 8 * bc.z + (li >> 6);
    const float x = (float)vx * nu, y = (float)vy * nu, z = (float)vz * nu;
    uint16_t *cnt = m.counts + (size_t)slot * L * kBlockVoxels + li;
    int fl = m.fused[vi];
    const int fl_in = fl;
    int votes = 0;
    for (int base = 0; base < cs.n; base += kCamChunk) {  // chunks in camera order
        int lab[kCamChunk];
#pragma unroll
        for (int k = 0; k < kCamChunk; ++k) {
            lab[k] = -1;
            const int ci = base + k;
            if (ci >= cs.n) continue;
            const Pose &T = cs.T[ci];
            const Camera &cam = cs.cam[ci];
            const float dx = x - T.m[3], dy = y - T.m[7], dz = z - T.m[11];
            const float px = (T.m[0] * dx + T.m[4] * dy) + T.m[8] * dz;
            const float py = (T.m[1] * dx + T.m[5] * dy) + T.m[9] * dz;
            const float pz = (T.m[2] * dx + T.m[6] * dy) + T.m[10] * dz;
            if (!(pz > 0.0f)) continue;
            const float u = cam.fx * (px / pz) + cam.cx;
            const float v = cam.fy * (py / pz) + cam.cy;
            if (!(u >= 0.0f && u < (float)cam.width && v >= 0.0f && v < (float)cam.height)) continue;
            lab[k] = cs.img[ci][(size_t)(int)v * cam.width + (int)u];
        }
        unsigned c0[kCamChunk];  // count of each camera's label before this chunk
#pragma unroll
        for (int k = 0; k < kCamChunk; ++k) {
            if (lab[k] >= L) lab[k] = -1;
            c0[k] = lab[k] >= 0 ? cnt[(size_t)lab[k] * kBlockVoxels] : 0u;
        }
        const int flc = fl;
        const unsigned cf0 = flc == 255 ? 0u : cnt[(size_t)flc * kBlockVoxels];
        unsigned cn[kCamChunk];  // count of camera k's label right after its vote
#pragma unroll
        for (int k = 0; k < kCamChunk; ++k) {
            cn[k] = 0;
            const int l = lab[k];
            if (l < 0) continue;
            unsigned cl = c0[k];
#pragma unroll
            for (int p = 0; p < k; ++p)
                if (lab[p] == l) cl = cn[p];  // latest earlier vote for the same label
            if (cl < 65535u) cl++;
            cn[k] = cl;
            unsigned cf = 0;
            if (fl != 255) {
                cf = fl == flc ? cf0 : 0u;
#pragma unroll
                for (int p = 0; p <= k; ++p)
                    if (lab[p] == fl) cf = cn[p];
            }
            if (l != fl && (cl > cf || (cl == cf && l < fl))) fl = l;
            votes++;
        }
#pragma unroll
        for (int k = 0; k < kCamChunk; ++k) {
            if (lab[k] < 0) continue;
            bool last = true;  // the last vote for this label writes its count
#pragma unroll
            for (int q = k + 1; q < kCamChunk; ++q)
                if (lab[q] == lab[k]) last = false;
            if (last) cnt[(size_t)lab[k] * kBlockVoxels] = (uint16_t)cn[k];
        }
    }
    if (fl != fl_in) m.fused[vi] = (uint8_t)fl;
    return votes;
}

// Pixel (floor u, floor v) of the voxel centre x under a pinhole camera at pose T, as a
// flat index into the image, or -1 when the voxel is behind the camera or off the image.
__device__ __forceinline__ long long camera_pixel(const Camera &cam, const Pose &T, float x, float y, float z)
{
    const float dx = x - T.m[3], dy = y - T.m[7], dz = z - T.m[11];
    const float px = (T.m[0] * dx + T.m[4] * dy) + T.m[8] * dz;
    const float py = (T.m[1] * dx + T.m[5] * dy) + T.m[9] * dz;
    const float pz = (T.m[2] * dx + T.m[6] * dy) + T.m[10] * dz;
    if (!(pz > 0.0f)) return -1;
    const float u = cam.fx * (px / pz) + cam.cx;
    const float v = cam.fy * (py / pz) + cam.cy;
    if (!(u >= 0.0f && u < (float)cam.width && v >= 0.0f && v < (float)cam.height)) return -1;
    return (long long)(int)v * cam.width + (int)u;
}

// The latest label wins (the paper's Ours-wo-Bay ablation, Sec. V-C): a band voxel takes
// the label of its latest observation, the last camera of the set that sees it with a
// label below L; vote counts are untouched.  Returns the votes.
__device__ __forceinline__ int label_voxel_latest(const MapView &m, const CameraSet &cs, int slot, int3 bc, int li)
{
    const size_t vi = (size_t)slot * kBlockVoxels + li;
    const float nu = m.nu;
    const int vx = 8 * bc.x + (li & 7), vy = 8 * bc.y + ((li >> 3) & 7), vz = 8 * bc.z + (li >> 6);
    const float x = (float)vx * nu, y = (float)vy * nu, z = (float)vz * nu;
    int lab = -1, votes = 0;
    for (int ci = 0; ci < cs.n; ++ci) {
        const long long q = camera_pixel(cs.cam[ci], cs.T[ci], x, y, z);
        if (q < 0) continue;
        const int l = cs.img[ci][q];
        if (l >= m.n_classes) continue;
        lab = l;
        votes++;
    }
    if (lab >= 0) m.fused[vi] = (uint8_t)lab;
    return votes;
}

// Eq. 6 on a camera's per-pixel class log-probabilities o (logp [height][width][L]): a
// band voxel seen at pixel q adds o(q) to its class log-posteriors and subtracts the
// largest sum (the normaliser Z, which keeps the posterior's ratios and argmax and needs
// no transcendental function); its most probable label is the class left at 0, the
// lowest on ties.  Up to kLpRegs classes are held in registers between the two passes;
// larger L recomputes the sums (the same fp32 values).  Returns 1 if the voxel voted.
constexpr int kLpRegs = 32;
__device__ __forceinline__ int logprob_voxel(const MapView &m, const Camera &cam, const Pose &T,
                                             const float *__restrict__ logp, int slot, int3 bc, int li)
{
    const float nu = m.nu;
    const int L = m.n_classes;
    const int vx = 8 * bc.x + (li & 7), vy = 8 * bc.y + ((li >> 3) & 7), vz = 8 * bc.z + (li >> 6);
    const long long q = camera_pixel(cam, T, (float)vx * nu, (float)vy * nu, (float)vz * nu);
    if (q < 0) return 0;
    const float *o = logp + (size_t)q * L;
    float *lp = m.logpost + (size_t)slot * L * kBlockVoxels + li;
    float mx = -INFINITY;
    int best = -1;
    if (L <= kLpRegs) {
        float s[kLpRegs];
#pragma unroll
        for (int l = 0; l < kLpRegs; ++l) {
            s[l] = 0.0f;
            if (l < L) s[l] = lp[(size_t)l * kBlockVoxels] + o[l];
        }
#pragma unroll
        for (int l = 0; l < kLpRegs; ++l)
            if (l < L && s[l] > mx) mx = s[l];
#pragma unroll
        for (int l = 0; l < kLpRegs; ++l) {
            if (l >= L) continue;
            const float d = s[l] - mx;
            lp[(size_t)l * kBlockVoxels] = d;
            if (best < 0 && d == 0.0f) best = l;
        }
    } else {
        for (int l = 0; l < L; ++l) {
            const float sl = lp[(size_t)l * kBlockVoxels] + o[l];
            if (sl > mx) mx = sl;
        }
        for (int l = 0; l < L; ++l) {
            const float d = (lp[(size_t)l * kBlockVoxels] + o[l]) - mx;
            lp[(size_t)l * kBlockVoxels] = d;
            if (best < 0 && d == 0.0f) best = l;
        }
    }
    m.fused[(size_t)slot * kBlockVoxels + li] = (uint8_t)best;
    return 1;
}

// Label fusion from a label range image (the scan's points labelled by a point-cloud
// segmentation): voxel li of the block at bc (slot `slot`) takes the label at its nearest
// pixel of the scan model under pose T (the pixel rule of the projective update) and votes
// with the rule of the camera labels (kLatest: the latest label wins).  Returns 1 if it
// voted.
template <bool kLatest = false>
__device__ __forceinline__ int label_voxel_lidar(const MapView &m, const LidarLUT &L, const Pose &T,
                                                 const uint8_t *__restrict__ img, int slot, int3 bc, int li)
{
    const float nu = m.nu;
    const int vx = 8 * bc.x + (li & 7), vy = 8 * bc.y + ((li >> 3) & 7), vz = 8 * bc.z + (li >> 6);
    const float x = (float)vx * nu, y = (float)vy * nu, z = (float)vz * nu;
    const float dx = x - T.m[3], dy = y - T.m[7], dz = z - T.m[11];
    const float px = (T.m[0] * dx + T.m[4] * dy) + T.m[8] * dz;
    const float py = (T.m[1] * dx + T.m[5] * dy) + T.m[9] * dz;
    const float pz = (T.m[2] * dx + T.m[6] * dy) + T.m[10] * dz;
    int row, col;
    if (!nearest_pixel(L, px, py, pz, row, col)) return 0;
    const int l = img[(size_t)row * L.cols + col];
    if (l >= m.n_classes) return 0;
    const size_t vi = (size_t)slot * kBlockVoxels + li;
    if (kLatest) {
        m.fused[vi] = (uint8_t)l;
        return 1;
    }
    uint16_t *cnt = m.counts + (size_t)slot * m.n_classes * kBlockVoxels + li;
    unsigned c = cnt[(size_t)l * kBlockVoxels];
    if (c < 65535u) c++;
    cnt[(size_t)l * kBlockVoxels] = (uint16_t)c;
    const int fl = m.fused[vi];
    const unsigned cf = fl == 255 ? 0u : (fl == l ? c : (unsigned)cnt[(size_t)fl * kBlockVoxels]);
    if (l != fl && (c > cf || (c == cf && l < fl))) m.fused[vi] = (uint8_t)l;
    return 1;
}

// ---------------------------------------------------------------------------------
// marching cubes of one block by one workgroup (see k_mesh.hip)
// ---------------------------------------------------------------------------------

__device__ __forceinline__ int halo_index(int x, int y, int z) { return x + kHalo * (y + kHalo * z); }

// local base corner of cube edge e (axis e / 4, the other two offsets from e % 4)
__device__ __forceinline__ int3 edge_base(int e)
{
    const int ax = e >> 2, j = e & 3;
    if (ax == 0) return make_int3(0, j & 1, j >> 1);
    if (ax == 1) return make_int3(j & 1, 0, j >> 1);
    return make_int3(j & 1, j >> 1, 0);
}

struct MeshLds {
    float2 dw[kHaloVoxels];
    uint8_t fused[kHaloVoxels];
    int nb[8];
    int wsum[kThreads / 64];
    unsigned long long base;
};

}  // namespace mc
