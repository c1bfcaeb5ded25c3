// Marching cubes of 8^3 blocks (end of Sec. IV-C.3), in two passes over the same
// candidate blocks: a counting pass (triangles per workgroup, from the voxel masks) and an
// emitting pass that writes each block's triangles at its offset, the prefix of those
// counts (summed by each emitting workgroup itself, or by a scan launch in batched
// steps).  No triangle reservation takes a shared atomic.  A worker (a workgroup, or a
// wavefront) stages a block and its +1 halo (9^3 voxels of distance, weight and fused
// label) in LDS from up to eight blocks, classifies the 512 cubes from the generated case
// table, and emits vertices on the sign-change edges.
#pragma once
#include "device.h"
#include "mc_table.inc"

namespace mc {

// A staged halo.  rows[y + 9 z] holds the sign bits (bits 0-8, D < 0) and observed bits
// (bits 16-24, W > 0) of the 9 voxels of x-row (y, z), so a cube's case comes from four
// row words.  The counting pass builds the rows from the voxel masks of the eight blocks
// (kept by the TSDF pass, 128 bytes per block); the emitting pass stages D and the fused
// label for the vertices, and per voxel a code byte (bit 0: D < 0, bit 1: W > 0) for the
// workgroup schedule's cube cases.
constexpr int kHaloRows = kHalo * kHalo;
struct HaloMask {
    unsigned long long mk[8][16];  // voxel masks of the blocks b + e (zero when absent)
    uint32_t rows[kHaloRows];
};
struct HaloFull {
    float d[kHaloVoxels];
    uint8_t code[kHaloVoxels];
    uint8_t fused[kHaloVoxels];
    uint32_t rows[kHaloRows];
};

// Candidates are meshed in batches of kMeshBatch blocks; a batch's block coordinates and
// neighbour slots are looked up by the whole workgroup at once (eight lanes per block)
// before any block of the batch is staged.
constexpr int kMeshBatch = kThreads / 8;
// Counting workgroups per emitting workgroup whose records an emitting workgroup reads.
constexpr int kMaxRecParts = 16;

// LDS of a meshing workgroup: the case tables (read per cube and per vertex, so they
// are copied from global memory once per workgroup; the counting pass needs only the
// triangle counts), one halo per worker, the iteration's candidate list and per-wave
// counts.
constexpr int kTriRow = 3 * MC_MAX_TRIS;
template <int kSched, class Halo>
struct __align__(16) MeshSmem {
    static constexpr bool kEmit = sizeof(Halo) == sizeof(HaloFull);  // the emitting pass's LDS
    uint8_t ntri[256];
    int8_t tris[sizeof(Halo) == sizeof(HaloFull) ? 256 * kTriRow : 4];
    Halo h[kSched == 0 ? 1 : kThreads / 64];
    uint8_t ccase[kSched == 0 ? 1 : kThreads / 64][sizeof(Halo) == sizeof(HaloFull) ? kBlockVoxels : 4];  // emitting
    int4 rbc[kThreads / 64];                                        // block of each worker in a round
    int4 bcs[kMeshBatch];
    int nbs[kMeshBatch][8];
    int mis[kMeshBatch];  // map of each batch entry (batched steps)
    int list[kThreads];
    int4 lbc[kEmit ? 1 : kThreads];  // counting pass: the candidates' coordinates
    int bt[kMeshBatch];              // counting pass: triangles of each block of a batch
    int rpre[kMaxRecParts + 1];      // emitting pass: prefix of its counting workgroups' records
    int wcnt[kThreads / 64];
    long long rcnt[kThreads / 64];
};

// The case tables reach the workgroup's LDS in two steps: every thread loads its dwords
// (t, t + kThreads, ...) into registers before the first candidate scan, so that the two
// loads overlap, and stores them after it; the scan's and the lookup's barriers order the
// stores before any cube is classified.  The counting pass needs only the triangle counts.
constexpr int kTabDwords = (256 + 256 * kTriRow) / 4;
constexpr int kTabPer = (kTabDwords + kThreads - 1) / kThreads;
struct TableRegs {
    uint32_t v[kTabPer];
};

template <bool kTris>
__device__ __forceinline__ TableRegs mesh_tables_load()
{
    const uint32_t *ntri = reinterpret_cast<const uint32_t *>(MC_NTRI);
    const uint32_t *tris = reinterpret_cast<const uint32_t *>(MC_TRIS);
    TableRegs r;
#pragma unroll
    for (int k = 0; k < kTabPer; ++k) {
        const int i = threadIdx.x + k * kThreads;
        r.v[k] = 0;
        if (i < 64) r.v[k] = ntri[i];
        else if (kTris && i < kTabDwords) r.v[k] = tris[i - 64];
    }
    return r;
}

template <bool kTris, class Smem>
__device__ __forceinline__ void mesh_tables_store(Smem &S, const TableRegs &r)
{
    uint32_t *ntri_s = reinterpret_cast<uint32_t *>(S.ntri);
    uint32_t *tris_s = reinterpret_cast<uint32_t *>(S.tris);
#pragma unroll
    for (int k = 0; k < kTabPer; ++k) {
        const int i = threadIdx.x + k * kThreads;
        if (i < 64) ntri_s[i] = r.v[k];
        else if (kTris && i < kTabDwords) tris_s[i - 64] = r.v[k];
    }
}

__device__ __forceinline__ void wave_lds_sync() { __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront"); }

template <int kSched>
__device__ __forceinline__ void worker_sync()
{
    if (kSched == 0) __syncthreads();
    else wave_lds_sync();
}

// Coordinates and neighbour slots (b + e, e in {0,1}^3; -1 when absent) of list entries
// j0 .. j0 + nb - 1, nb <= kMeshBatch; every thread calls it.  The counting pass has the
// coordinates from its candidate scan, looks the neighbours up in the hash and keeps them
// in mesh_nbr for the emitting pass, which fetches them with one coalesced read per block.
template <class Smem>
__device__ __forceinline__ void mesh_batch_lookup(const MapView &m, Smem &S, int j0, int nb)
{
    const int jb = threadIdx.x >> 3, e = threadIdx.x & 7;
    if (jb < nb) {
        const int slot = S.list[j0 + jb];
        int s;
        if constexpr (Smem::kEmit) {
            s = m.mesh_nbr[(size_t)slot * 8 + e];
            if (e == 0) S.bcs[jb] = m.coords[slot];
        } else {
            const int4 bc = S.lbc[j0 + jb];  // read by the candidate scan
            s = e == 0 ? slot : hash_find(m, pack_key(bc.x + (e & 1), bc.y + ((e >> 1) & 1), bc.z + ((e >> 2) & 1)));
            m.mesh_nbr[(size_t)slot * 8 + e] = s;
        }
        S.nbs[jb][e] = s;
    }
    __syncthreads();
}

__device__ __forceinline__ uint8_t voxel_code(float2 v)
{
    return (uint8_t)((v.x < 0.0f ? 1 : 0) | (v.y > 0.0f ? 2 : 0));
}

// Stage the halo of the block whose neighbour slots are nb[8] (absent blocks are
// unobserved); rank is the lane's index among the worker's kWidth.
template <int kSched>
__device__ __forceinline__ void mesh_stage(const MapView &m, const int *nb, HaloFull &S, int rank)
{
    constexpr int kWidth = kSched == 0 ? kThreads : 64;
    for (int h = rank; h < kHaloVoxels; h += kWidth) {
        const int hx = h % kHalo, hy = (h / kHalo) % kHalo, hz = h / (kHalo * kHalo);
        const int s = nb[(hx >> 3) | ((hy >> 3) << 1) | ((hz >> 3) << 2)];
        if (s >= 0) {
            const size_t vi = (size_t)s * kBlockVoxels + (hx & 7) + 8 * (hy & 7) + 64 * (hz & 7);
            const float2 v = m.dw[vi];
            S.d[h] = v.x;
            S.code[h] = voxel_code(v);
            S.fused[h] = m.fused[vi];
        } else {
            S.d[h] = 0.0f;
            S.code[h] = 0;
            S.fused[h] = 255;
        }
    }
    worker_sync<kSched>();
}

// Stage a halo by rows (one wavefront): lane l takes rows l and l + 64.  A row's 8
// voxels of one block are 64 contiguous bytes (four 16-byte loads), the 9th is the first
// voxel of the +x neighbour's row; both blocks' loads are issued before either is used,
// so a row costs one memory round trip.  The row's D values and fused labels are staged
// too (halo index x + 9 row).
__device__ __forceinline__ void mesh_stage_rows(const MapView &m, const int *nb, HaloFull &S, int lane)
{
    for (int r = lane; r < kHaloRows; r += 64) {
        const int y = r % kHalo, z = r / kHalo;
        const int jj = ((y >> 3) << 1) | ((z >> 3) << 2);
        const int s0 = nb[jj], s1 = nb[jj | 1];
        const int off = 8 * (y & 7) + 64 * (z & 7);
        // branch-free loads (an absent block reads slot 0 and is then masked out), so the
        // compiler issues all of them before the first use
        const size_t v0 = (size_t)(s0 >= 0 ? s0 : 0) * kBlockVoxels + off;
        const size_t v1 = (size_t)(s1 >= 0 ? s1 : 0) * kBlockVoxels + off;
        float4 q[4];
        const float4 *p = reinterpret_cast<const float4 *>(m.dw + v0);
#pragma unroll
        for (int i = 0; i < 4; ++i) q[i] = p[i];
        unsigned long long f8 = *reinterpret_cast<const unsigned long long *>(m.fused + v0);
        float2 v9 = m.dw[v1];
        uint8_t u9 = m.fused[v1];
        if (s0 < 0) {  // absent: unobserved, fused 255
#pragma unroll
            for (int i = 0; i < 4; ++i) q[i] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            f8 = ~0ull;
        }
        if (s1 < 0) {
            v9 = make_float2(0.0f, 0.0f);
            u9 = 255;
        }
        uint32_t sign = 0, obs = 0;
        const int h = kHalo * r;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const float D0 = q[i].x, W0 = q[i].y, D1 = q[i].z, W1 = q[i].w;
            sign |= (D0 < 0.0f ? 1u : 0u) << (2 * i) | (D1 < 0.0f ? 1u : 0u) << (2 * i + 1);
            obs |= (W0 > 0.0f ? 1u : 0u) << (2 * i) | (W1 > 0.0f ? 1u : 0u) << (2 * i + 1);
            S.d[h + 2 * i] = D0;
            S.d[h + 2 * i + 1] = D1;
        }
        sign |= (v9.x < 0.0f ? 1u : 0u) << 8;
        obs |= (v9.y > 0.0f ? 1u : 0u) << 8;
        S.d[h + 8] = v9.x;
#pragma unroll
        for (int x = 0; x < 8; ++x) S.fused[h + x] = (uint8_t)(f8 >> (8 * x));
        S.fused[h + 8] = u9;
        S.rows[r] = sign | (obs << 16);
    }
    wave_lds_sync();
}

// Stage a block's halo rows from the voxel masks of its eight blocks (one wavefront):
// lane l copies 16 bytes of block l / 8's masks into LDS, then builds rows l and l + 64.
__device__ __forceinline__ void mesh_stage_masks(const MapView &m, const int *nb, HaloMask &S, int lane)
{
    const int jj = lane >> 3, q = lane & 7;
    const int s = nb[jj];
    ulonglong2 v = make_ulonglong2(0ull, 0ull);
    if (s >= 0) v = reinterpret_cast<const ulonglong2 *>(m.vmask + (size_t)s * 16)[q];
    reinterpret_cast<ulonglong2 *>(S.mk[jj])[q] = v;
    wave_lds_sync();
    for (int r = lane; r < kHaloRows; r += 64) {
        const int y = r % kHalo, z = r / kHalo;
        const int j0 = ((y >> 3) << 1) | ((z >> 3) << 2);
        const int sl = z & 7, sh = 8 * (y & 7);
        const uint32_t sign = (uint32_t)((S.mk[j0][sl] >> sh) & 0xFFu) | (uint32_t)((S.mk[j0 | 1][sl] >> sh) & 1u) << 8;
        const uint32_t obs =
            (uint32_t)((S.mk[j0][8 + sl] >> sh) & 0xFFu) | (uint32_t)((S.mk[j0 | 1][8 + sl] >> sh) & 1u) << 8;
        S.rows[r] = sign | (obs << 16);
    }
    wave_lds_sync();
}

// Cases of the lane's 8 cubes, the x-row (cy, cz) = (lane % 8, lane / 8): cube cx has
// index cx + 8 lane.  Returns the lane's triangles, packs each cube's count into 4 bits of
// *counts (cube cx in nibble cx) and stores its case in ccase when given.
template <class Halo>
__device__ __forceinline__ int mesh_classify_rows(const Halo &S, const uint8_t *ntri, int lane, uint8_t *ccase,
                                                  unsigned *counts)
{
    const int cy = lane & 7, cz = lane >> 3;
    const uint32_t r00 = S.rows[cy + kHalo * cz], r10 = S.rows[cy + 1 + kHalo * cz];
    const uint32_t r01 = S.rows[cy + kHalo * (cz + 1)], r11 = S.rows[cy + 1 + kHalo * (cz + 1)];
    int mine = 0;
    unsigned packed = 0;
#pragma unroll
    for (int cx = 0; cx < 8; ++cx) {
        const uint32_t k = ((r00 >> cx) & 3u) | (((r10 >> cx) & 3u) << 2) | (((r01 >> cx) & 3u) << 4) |
                           (((r11 >> cx) & 3u) << 6);
        const uint32_t v = (r00 >> (16 + cx)) & (r10 >> (16 + cx)) & (r01 >> (16 + cx)) & (r11 >> (16 + cx)) & 3u;
        const int nt = v == 3u ? (int)ntri[k] : 0;
        if (ccase) ccase[cx + 8 * lane] = (uint8_t)k;
        packed |= (unsigned)nt << (4 * cx);
        mine += nt;
    }
    *counts = packed;
    return mine;
}

// Cases of the lane's cubes (cube it * kWidth + rank): returns the lane's triangles,
// packs each cube's triangle count into 4 bits of *counts, and stores each cube's case
// in ccase[cube] when ccase is given.  A cube counts only when all eight corners are
// observed (W > 0).
template <int kSched, class Halo>
__device__ __forceinline__ int mesh_classify(const Halo &S, const uint8_t *ntri, int rank, uint8_t *ccase,
                                             unsigned *counts)
{
    constexpr int kWidth = kSched == 0 ? kThreads : 64;
    constexpr int kCubes = kBlockVoxels / kWidth;
    int mine = 0;
    unsigned packed = 0;
#pragma unroll
    for (int it = 0; it < kCubes; ++it) {
        const int cube = it * kWidth + rank;
        const int cx = cube & 7, cy = (cube >> 3) & 7, cz = cube >> 6;
        int valid = 2, k = 0;
#pragma unroll
        for (int n = 0; n < 8; ++n) {
            const int c = S.code[halo_index(cx + (n & 1), cy + ((n >> 1) & 1), cz + ((n >> 2) & 1))];
            valid &= c;
            k |= (c & 1) << n;
        }
        const int nt = valid ? (int)ntri[k] : 0;
        if (ccase) ccase[cube] = (uint8_t)k;
        packed |= (unsigned)nt << (4 * it);
        mine += nt;
    }
    *counts = packed;
    return mine;
}

// Triangles are emitted a window of kStageTris at a time: each thread finds the cube and
// triangle of one window index from the round's per-lane start indices and packed cube
// counts (a binary search over the workgroup's lanes, then a walk over the lane's cubes)
// and writes that whole triangle to its output index.  Consecutive threads write
// consecutive triangles, so the caches merge the stores; staging the window in LDS for
// contiguous stores took 10 KB of LDS (four emitting workgroups per compute unit instead
// of five) and two barriers a window, and measured 3 us slower per street frame.
constexpr int kStageTris = 256;
struct MeshStage {
    int lo[kThreads];        // first round index of each lane's triangles
    unsigned cnt[kThreads];  // each lane's cube triangle counts, 4 bits per cube
};

// Build the triangle with descriptor d (worker << 12 | cube << 3 | triangle of the cube)
// at output index g: positions, labels and, when asked for, edge keys (indices at or past
// out.cap are dropped: the extraction then reports the size it needs).
template <class Smem>
__device__ __forceinline__ void mesh_tri(const MapView &m, const Smem &S, int d, long long g, const MeshOut &out)
{
    const int wk = d >> 12, cube = (d >> 3) & 511, q = d & 7;
    const HaloFull &H = S.h[wk];
    const int4 bc = S.rbc[wk];
    const int8_t *row = S.tris + (int)S.ccase[wk][cube] * kTriRow + 3 * q;
    const int cx = cube & 7, cy = (cube >> 3) & 7, cz = cube >> 6;
    const float nu = m.nu;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const int ed = row[k];
        const int ax = ed >> 2;
        const int3 o = edge_base(ed);
        const int ax_ = cx + o.x, ay_ = cy + o.y, az_ = cz + o.z;
        const int ha = halo_index(ax_, ay_, az_);
        const int hb = halo_index(ax_ + (ax == 0), ay_ + (ax == 1), az_ + (ax == 2));
        const float Da = H.d[ha], Db = H.d[hb];
        const float tt = Da / (Da - Db);
        const int vx = 8 * bc.x + ax_, vy = 8 * bc.y + ay_, vz = 8 * bc.z + az_;
        float P[3] = {(float)vx * nu, (float)vy * nu, (float)vz * nu};
        P[ax] = P[ax] + tt * nu;
        if (g < out.cap) {
            out.pos[g * 9 + 3 * k] = P[0];
            out.pos[g * 9 + 3 * k + 1] = P[1];
            out.pos[g * 9 + 3 * k + 2] = P[2];
            out.lab[g * 3 + k] = fabsf(Da) <= fabsf(Db) ? H.fused[ha] : H.fused[hb];
        }
        if (out.ekey && g < out.cap) {
            const long long off = 1LL << 19;
            out.ekey[g * 3 + k] = ((vx + off) << 42) | ((vy + off) << 22) | ((vz + off) << 2) | ax;
        }
    }
}

// One round's output (its blocks' triangles are contiguous from output index r0): the
// lane's triangles are [lo, lo + mine) within the round of rtot; every thread of the
// workgroup calls it.  Lane start indices never decrease with the thread index, so the
// last lane whose start is at most i is the one that holds round index i.
template <int kSched, class Smem>
__device__ __forceinline__ void mesh_round_out(const MapView &m, const Smem &S, MeshStage &st, bool has,
                                               unsigned counts, int lo, int rtot, long long r0, const MeshOut &out)
{
    constexpr int kWidth = kSched == 0 ? kThreads : 64;
    constexpr int kCubes = kBlockVoxels / kWidth;
    st.lo[threadIdx.x] = lo;
    st.cnt[threadIdx.x] = has ? counts : 0u;
    __syncthreads();
    for (int w0 = 0; w0 < rtot; w0 += kStageTris) {
        const int nw = rtot - w0 < kStageTris ? rtot - w0 : kStageTris;
        const int i = threadIdx.x;
        if (i < nw) {
            const int g = w0 + i;
            int T = 0;
#pragma unroll
            for (int step = kThreads / 2; step > 0; step >>= 1)
                if (st.lo[T + step] <= g) T += step;
            const unsigned c = st.cnt[T];
            int local = g - st.lo[T], it_hit = 0, q = 0;
            bool found = false;
#pragma unroll
            for (int it = 0; it < kCubes; ++it) {
                const int nt = (int)((c >> (4 * it)) & 15u);
                if (!found && local < nt) {
                    found = true;
                    it_hit = it;
                    q = local;
                }
                local -= found ? 0 : nt;
            }
            const int worker = kSched == 0 ? 0 : T >> 6, rank = kSched == 0 ? T : T & 63;
            const int cube = kSched == 0 ? it_hit * kWidth + rank : it_hit + 8 * rank;  // the rows' cube order
            mesh_tri(m, S, (worker << 12) | (cube << 3) | q, r0 + g, out);
        }
    }
}

// Inclusive wavefront scan.
__device__ __forceinline__ int wave_scan_incl(int v)
{
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int y = __shfl_up(v, off, 64);
        if (lane >= off) v += y;
    }
    return v;
}

// The counting pass's candidates: the map's slots [0, nslots), dealt out one at a time,
// thread t of workgroup w taking slot (q kThreads + t) G + w in round q, so that a cluster
// of dirty slots spreads over all workgroups.  A slot is taken if `all` or its dirty mark
// (coordinates .w) holds `epoch`.  Candidates reach the workgroup kThreads at a time,
// compacted into S.list (slots) and S.lbc (coordinates).

// Keep the round's slots that pass (one per thread), compacted in thread order; returns
// their number.  The caller's reads of S.list are complete (a barrier follows the ballot).
template <class Smem>
__device__ __forceinline__ int mesh_take(bool take, int slot, int4 bc, Smem &S)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const unsigned long long bal = __ballot(take);
    if (lane == 0) S.wcnt[wave] = __popcll(bal);
    __syncthreads();
    int off = 0, n = 0;
#pragma unroll
    for (int w = 0; w < kThreads / 64; ++w) {
        const int c = S.wcnt[w];
        off += w < wave ? c : 0;
        n += c;
    }
    if (take) {
        const int at = off + __popcll(bal & ((1ull << lane) - 1ull));
        S.list[at] = slot;
        S.lbc[at] = bc;
    }
    __syncthreads();
    return n;
}

// Sweep of the slots: round `it`'s dirty candidates (or all of them), or -1 past the end.
// The coordinates are read for every slot (their .w is the dirty mark).
template <class Smem>
__device__ __forceinline__ int mesh_candidates(const MapView &m, bool all, uint32_t epoch, int nslots, int it, Smem &S)
{
    if (((long long)it * kThreads * gridDim.x + blockIdx.x) >= nslots) return -1;
    const long long slot = ((long long)it * kThreads + threadIdx.x) * gridDim.x + blockIdx.x;
    bool take = false;
    int4 bc = make_int4(0, 0, 0, 0);
    if (slot < nslots) {
        bc = m.coords[slot];
        take = all || (uint32_t)bc.w == epoch;
    }
    return mesh_take(take, (int)slot, bc, S);
}

// From the dirty bitmap instead (a DIRTY extraction of a large map): the workgroup's
// slots w + j G are bits j of its own words of the bitmap, so thread t reads word t (bits
// j = 32 t ...) and clears it, and the candidates cost one bitmap word per 32 slots and one
// coordinate read per marked block, not a coordinate read per allocated slot.  Candidate i
// of the workgroup (marked slots in j order, as the sweep would take them) goes to chunk
// i / kThreads.  One word per thread: pools up to 8192 G blocks.
struct BitCands {
    uint32_t mask;  // bit b: slot w + (32 t + b) G is marked
    int base;       // index of this thread's first candidate in the workgroup
    int total;      // the workgroup's candidates
};

__device__ __forceinline__ BitCands mesh_bits_take(const MapView &m, int nslots, int *s_tmp)
{
    const int G = (int)gridDim.x, w = (int)blockIdx.x, t = (int)threadIdx.x;
    const int nj = nslots > w ? (nslots - w + G - 1) / G : 0;  // the workgroup's slots
    uint32_t mask = 0;
    if (t < (nj + 31) >> 5) {
        uint32_t *word = &m.dbits[(size_t)w * m.bits_wpw + t];
        mask = *word;
        const int left = nj - 32 * t;  // slots of this word (bits past them are never set)
        if (left < 32) mask &= (1u << left) - 1u;
        *word = 0u;  // a thread's load and later store of one address keep their order
    }
    BitCands b;
    b.mask = mask;
    b.base = wg_scan(__popc(mask), s_tmp, &b.total);
    return b;
}

template <class Smem>
__device__ __forceinline__ int mesh_candidates_bits(const MapView &m, const BitCands &b, uint32_t epoch, int it,
                                                    Smem &S)
{
    const int lo = it * kThreads;
    if (lo >= b.total) return -1;
    const long long G = gridDim.x;
    uint32_t x = b.mask;
    for (int idx = b.base; x && idx < lo + kThreads; ++idx) {  // this thread's candidates of the chunk
        const int bit = __ffs(x) - 1;
        x &= x - 1u;
        if (idx >= lo) S.list[idx - lo] = (int)(blockIdx.x + (32ll * threadIdx.x + bit) * G);
    }
    __syncthreads();
    const int n = b.total - lo < kThreads ? b.total - lo : kThreads;
    const bool has = (int)threadIdx.x < n;
    const int slot = has ? S.list[threadIdx.x] : 0;
    const int4 bc = m.coords[slot];  // branch-free: slot 0 for threads past the chunk, unused
    return mesh_take(has && (uint32_t)bc.w == epoch, slot, bc, S);  // a bit may outlive its mark
}

// Counting pass of one workgroup: triangles and blocks over its candidates, one
// wavefront per block (halo rows from the voxel masks).  With rec (per-map extractions),
// the blocks with triangles are recorded in candidate order (coordinates, slot, neighbour
// slots) and their number is written to *nz, so the emitting pass reads them directly.
__device__ __forceinline__ void mesh_count_wg(const MapView &m, bool all, uint32_t epoch, int nslots,
                                              MeshSmem<1, HaloMask> &S, long long *tris, int *blocks,
                                              MeshRec *rec = nullptr, int32_t *nz = nullptr, int rec_cap = 0,
                                              bool bits = false)
{
    const TableRegs tab = mesh_tables_load<false>();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    long long my_tris = 0;
    int my_blocks = 0, n_rec = 0;
    unsigned counts;
    BitCands bcand{0u, 0, 0};
    if (bits) bcand = mesh_bits_take(m, nslots, S.wcnt);
    for (int it = 0;; ++it) {
        const int n = bits ? mesh_candidates_bits(m, bcand, epoch, it, S) : mesh_candidates(m, all, epoch, nslots, it, S);
        if (it == 0) mesh_tables_store<false>(S, tab);
        if (n < 0) break;
        for (int j0 = 0; j0 < n; j0 += kMeshBatch) {
            const int nb = n - j0 < kMeshBatch ? n - j0 : kMeshBatch;
            mesh_batch_lookup(m, S, j0, nb);
            for (int j = wave; j < nb; j += kThreads / 64) {
                mesh_stage_masks(m, S.nbs[j], S.h[wave], lane);
                const unsigned long long t =
                    wave_sum_u64((unsigned long long)mesh_classify_rows(S.h[wave], S.ntri, lane, nullptr, &counts));
                wave_lds_sync();
                if (lane == 0) {
                    m.mesh_cnt[S.nbs[j][0]] = (uint16_t)t;
                    my_tris += (long long)t;
                    my_blocks += 1;
                    S.bt[j] = (int)t;
                }
            }
            __syncthreads();
            if (rec) {  // the batch's blocks with triangles, appended in batch order by wave 0
                if (wave == 0) {
                    const bool has = lane < nb && S.bt[lane] > 0;
                    const unsigned long long bal = __ballot(has);
                    const int at = n_rec + __popcll(bal & ((1ull << lane) - 1ull));
                    if (has && at < rec_cap) {
                        int4 bc = S.lbc[j0 + lane];
                        bc.w = S.list[j0 + lane];
                        int4 *dst = reinterpret_cast<int4 *>(rec + at);
                        dst[0] = bc;
                        dst[1] = make_int4(S.nbs[lane][0], S.nbs[lane][1], S.nbs[lane][2], S.nbs[lane][3]);
                        dst[2] = make_int4(S.nbs[lane][4], S.nbs[lane][5], S.nbs[lane][6], S.nbs[lane][7]);
                    }
                    n_rec += __popcll(bal);
                }
                __syncthreads();  // the batch's lookups are rewritten by the next batch
            }
        }
        __syncthreads();  // the list is rewritten by the next iteration
    }
    if (rec && threadIdx.x == 0) *nz = n_rec;
    // workgroup totals (kept on lane 0 of each wavefront)
    unsigned long long t = wave_sum_u64((unsigned long long)my_tris);
    unsigned long long b = wave_sum_u64((unsigned long long)my_blocks);
    if (lane == 0) {
        S.rcnt[wave] = (long long)t;
        S.wcnt[wave] = (int)b;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        long long tt = 0;
        int bb = 0;
        for (int w = 0; w < kThreads / 64; ++w) {
            tt += S.rcnt[w];
            bb += S.wcnt[w];
        }
        *tris = tt;
        *blocks = bb;
    }
}

// Emitting pass of one per-map workgroup from the counting pass's records: the blocks of
// counting workgroups w + j G (j < k) in that order, batch by batch (each batch's records
// read at once into the lookup arrays), triangles from output index `base` on.  A round is
// one block (kSched 0) or one block per wave (kSched 1); a round's output is contiguous, in
// wave order.
template <int kSched>
__device__ __forceinline__ void mesh_emit_recs(const MapView &m, const MeshScan &scan, int k, int my_nz,
                                               long long base, const MeshOut &out, MeshSmem<kSched, HaloFull> &S,
                                               MeshStage &st, const TableRegs &tab)
{
    constexpr int kPerRound = kSched == 0 ? 1 : kThreads / 64;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int rank = kSched == 0 ? (int)threadIdx.x : lane;
    const int worker = kSched == 0 ? 0 : wave;
    const int G = (int)gridDim.x;
    if (wave == 0) {  // prefix of the record counts (thread j < k holds counting workgroup w + j G's)
        const int incl = wave_scan_incl(my_nz);
        if (lane < k) S.rpre[lane + 1] = incl;
        if (lane == 0) S.rpre[0] = 0;
    }
    mesh_tables_store<true>(S, tab);
    __syncthreads();
    const int total = S.rpre[k];
    unsigned counts = 0;
    long long carry = base;
    for (int j0 = 0; j0 < total; j0 += kMeshBatch) {
        const int nb = total - j0 < kMeshBatch ? total - j0 : kMeshBatch;
        {  // eight lanes per record: lane e of record jb reads its neighbour slot e (and e = 0 the block)
            const int jb = threadIdx.x >> 3, e = threadIdx.x & 7;
            if (jb < nb) {
                const int r = j0 + jb;
                int j = 0;
                for (int q = 1; q < k; ++q) j += S.rpre[q] <= r ? 1 : 0;
                const MeshRec *src = scan.rec + (size_t)(blockIdx.x + j * G) * scan.rec_cap + (r - S.rpre[j]);
                S.nbs[jb][e] = src->nb[e];
                if (e == 0) S.bcs[jb] = src->bc;
            }
            __syncthreads();
        }
        for (int r = 0; r < nb; r += kPerRound) {
            const int j = r + worker;
            const bool has = j < nb;
            int mine = 0;
            if (kSched == 0) {
                mesh_stage<0>(m, S.nbs[j], S.h[0], rank);
                if (rank == 0) S.rbc[0] = S.bcs[j];
                mine = mesh_classify<0>(S.h[0], S.ntri, rank, S.ccase[0], &counts);
            } else if (has) {
                mesh_stage_rows(m, S.nbs[j], S.h[worker], lane);
                if (lane == 0) S.rbc[worker] = S.bcs[j];
                mine = mesh_classify_rows(S.h[worker], S.ntri, lane, S.ccase[worker], &counts);
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
            mesh_round_out<kSched>(m, S, st, has, counts, woff + incl - mine, rtot, carry, out);
            carry += rtot;
            __syncthreads();  // the round's counts are rewritten by the next round
        }
    }
}

// The emitting workgroup's output offset, from the counting pass's per-workgroup counts:
// emitting workgroup w takes the slots of counting workgroups c with c mod G = w, so its
// offset sums the counts of those with c mod G < w.  Every thread calls it; the counts are
// read at once (thread t takes t + q kThreads), clamped and masked.  Workgroup 0 (offset
// 0) also sums every count and does the extraction's bookkeeping: totals, the epoch
// advance that clears the dirty set when a DIRTY extraction fits (the counting pass has
// read the epoch; the emitting pass meshes mesh_epoch, recorded by the counting pass),
// the dirty bitmap's gap flag (a DIRTY extraction that does not fit keeps the dirty set,
// which the counting pass may have cleared from the bitmap), and the host report, which
// therefore arrives while the rest of the pass still runs.
__device__ __forceinline__ long long mesh_emit_base(const MapView &m, int mode, const long long *wg_tris,
                                                    const int32_t *wg_blocks, int g_count, long long cap,
                                                    MeshReport *report, long long *s_red)
{
    constexpr int kPer = kMaxMeshGrid / kThreads;
    constexpr int kWaves = kThreads / 64;
    const int G = (int)gridDim.x, w = (int)blockIdx.x;
    const bool lead = w == 0;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    Counters *c = m.ctr;
    uint32_t epoch = 0, seq = 0;
    if (lead && threadIdx.x == 0) {
        epoch = c->dirty_epoch;
        seq = c->extractions + 1;
    }
    const float inv_g = 1.0f / (float)G;
    long long v[kPer];
    int b[kPer];
    bool need[kPer], before[kPer];
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
        const int cw = (int)threadIdx.x + q * kThreads;
        int r = cw - (int)((float)cw * inv_g) * G;  // cw mod G (the float quotient is off by at most one)
        r += r < 0 ? G : 0;
        r -= r >= G ? G : 0;
        before[q] = cw < g_count && r < w;
        need[q] = before[q] || (lead && cw < g_count);
        const int idx = need[q] ? cw : 0;
        v[q] = wg_tris[idx];
        b[q] = wg_blocks[lead ? idx : 0];  // branch-free (other workgroups read entry 0, unused)
    }
    long long part = 0, tot = 0, blk = 0;
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
        part += before[q] ? v[q] : 0;
        tot += need[q] ? v[q] : 0;
        blk += need[q] ? b[q] : 0;
    }
    part = (long long)wave_sum_u64((unsigned long long)part);
    if (lead) {
        tot = (long long)wave_sum_u64((unsigned long long)tot);
        blk = (long long)wave_sum_u64((unsigned long long)blk);
    }
    if (lane == 0) {
        s_red[wave] = part;
        s_red[kWaves + wave] = tot;
        s_red[2 * kWaves + wave] = blk;
    }
    __syncthreads();
    long long off = 0, total = 0, blocks = 0;
#pragma unroll
    for (int i = 0; i < kWaves; ++i) {
        off += s_red[i];
        total += s_red[kWaves + i];
        blocks += s_red[2 * kWaves + i];
    }
    if (lead && threadIdx.x == 0) {
        c->mesh_tris = (unsigned long long)total;
        c->mesh_blocks = (unsigned long long)blocks;
        if (mode == 0) {
            if (total <= cap) c->dirty_epoch = epoch + 1;
            c->bits_gap = total <= cap ? 0 : 1;  // a new epoch has no frame yet
        }
        c->extractions = seq;
        if (report) {  // host memory: system-scope stores; the host waits for seq
            __hip_atomic_store(&report->tris, (unsigned long long)total, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
            __hip_atomic_store(&report->blocks, (unsigned long long)blocks, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_SYSTEM);
            __hip_atomic_store(&report->seq, (unsigned long long)seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
        }
    }
    return off;
}

// Batched steps: exclusive scan of one map's counts per emitting workgroup (one workgroup): offsets,
// and the extraction's bookkeeping.  Emitting workgroup w covers counting workgroups
// w + j G, j < k; entry w of the arrays is at index w * stride.  A DIRTY extraction whose
// output fits clears the dirty set by advancing the epoch; the emitting pass meshes the
// epoch recorded here.
__device__ __forceinline__ void mesh_scan_map(const MapView &m, int mode, const long long *wg_tris,
                                              const int32_t *wg_blocks, long long *wg_off, int G, int k, int stride,
                                              long long cap, MeshReport *report)
{
    __shared__ long long s_part[kThreads / 64];
    __shared__ long long s_blk[kThreads / 64];
    constexpr int kPer = kMaxMeshGrid / kThreads;  // loads per thread: per * k <= kPer
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int per = (G + kThreads - 1) / kThreads;
    const int w0 = threadIdx.x * per;
    // thread t sums emitting workgroups w0 .. w0 + per - 1, k counting workgroups each: the
    // per * k counts are walked as (i, j) = (f / k, f mod k) in chunks of kPer loads issued
    // together (one chunk unless the emitting grid is far from a multiple of kThreads);
    // the first chunk's values are kept for the offsets
    const int nf = per * k;
    Counters *c = m.ctr;
    uint32_t epoch = 0, seq = 0;
    if (threadIdx.x == 0) {  // read with the counts: used after the scan
        epoch = c->dirty_epoch;
        seq = c->extractions + 1;
    }
    long long v[kPer];
    long long sum = 0, blk = 0;
    for (int f0 = 0; f0 < nf; f0 += kPer) {
        int i = f0 / k, j = f0 - (f0 / k) * k;
        long long t[kPer];
        int b[kPer];
#pragma unroll
        for (int f = 0; f < kPer; ++f) {
            const bool ok = f0 + f < nf && w0 + i < G;
            const size_t idx = ok ? (size_t)(w0 + i + j * G) * stride : 0;  // branch-free: entry 0, masked
            t[f] = wg_tris[idx];
            b[f] = wg_blocks[idx];
            t[f] = ok ? t[f] : 0;
            b[f] = ok ? b[f] : 0;
            if (++j == k) {
                j = 0;
                ++i;
            }
        }
#pragma unroll
        for (int f = 0; f < kPer; ++f) {  // no use before every load is issued
            sum += t[f];
            blk += b[f];
            if (f0 == 0) v[f] = t[f];
        }
    }
    long long incl = sum;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const long long y = __shfl_up(incl, off, 64);
        if (lane >= off) incl += y;
    }
    const unsigned long long bw = wave_sum_u64((unsigned long long)blk);
    if (lane == 63) s_part[wave] = incl;
    if (lane == 0) s_blk[wave] = (long long)bw;
    __syncthreads();
    long long before = 0, total = 0, blocks = 0;
#pragma unroll
    for (int w = 0; w < kThreads / 64; ++w) {
        before += w < wave ? s_part[w] : 0;
        total += s_part[w];
        blocks += s_blk[w];
    }
    long long run = before + incl - sum;
    {  // the first chunk from registers (no load between the offset stores)
        int i = 0, j = 0;
#pragma unroll
        for (int f = 0; f < kPer; ++f) {
            const bool ok = f < nf && w0 + i < G;
            if (ok && j == 0) wg_off[(size_t)(w0 + i) * stride] = run;
            run += ok ? v[f] : 0;
            if (++j == k) {
                j = 0;
                ++i;
            }
        }
    }
    for (int f0 = kPer; f0 < nf; f0 += kPer) {  // further chunks are read again
        int i = f0 / k, j = f0 - (f0 / k) * k;
        for (int f = 0; f < kPer; ++f) {
            const bool ok = f0 + f < nf && w0 + i < G;
            if (ok && j == 0) wg_off[(size_t)(w0 + i) * stride] = run;
            run += ok ? wg_tris[(size_t)(w0 + i + j * G) * stride] : 0;
            if (++j == k) {
                j = 0;
                ++i;
            }
        }
    }
    if (threadIdx.x == 0) {
        c->mesh_epoch = epoch;
        c->mesh_tris = (unsigned long long)total;
        c->mesh_blocks = (unsigned long long)blocks;
        if (mode == 0 && total <= cap) {
            c->dirty_epoch = epoch + 1;
            c->bits_gap = 0;  // a new epoch has no frame yet (set bits of older marks only cost work)
        }
        c->extractions = seq;
        if (report) {  // host memory: system-scope stores; the host waits for seq, so it
                       // can return while the emitting pass still runs
            __hip_atomic_store(&report->tris, (unsigned long long)total, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
            __hip_atomic_store(&report->blocks, (unsigned long long)blocks, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_SYSTEM);
            __hip_atomic_store(&report->seq, (unsigned long long)seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
        }
    }
}

// Workgroups of the counting and emitting passes: each as many as the device holds at
// once, the counting grid rounded down to a multiple of the emitting grid (emitting
// workgroup w takes the slots of counting workgroups w + j G_emit), so every
// workgroup's latency chain runs concurrently.
template <class CountK, class EmitK>
inline MeshGrid resident_grids(CountK count_k, EmitK emit_k)
{
    int dev = 0, cus = 0, a = 0, b = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&a, count_k, kThreads, 0) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, emit_k, kThreads, 0) != hipSuccess || cus < 1 || a < 1 ||
        b < 1)
        return MeshGrid{1024, 1024};
    long long ge = (long long)cus * b, gc = (long long)cus * a;
    if (ge > kMaxMeshGrid) ge = kMaxMeshGrid;
    if (gc > kMaxMeshGrid) gc = kMaxMeshGrid;
    if (gc < ge) gc = ge;
    gc -= gc % ge;
    return MeshGrid{(int)ge, (int)gc};
}

}  // namespace mc
