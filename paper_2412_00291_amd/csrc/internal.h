// Internal types shared by the mapcore HIP sources (device views, launch wrappers).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mc {

constexpr int kBlockVoxels = 512;
constexpr unsigned long long kEmpty = ~0ull;
constexpr int kFxShift = 16;                  // 2^-16 voxel fixed point
constexpr long long kBlockFx = 8LL << kFxShift;  // one block edge in fixed point
constexpr int kDomainVoxels = (1 << 19) - 64;    // |voxel index| bound of the map domain

// Device-side counters of one map.  Per-frame counters are reset on the device by the
// last workgroup of the TSDF kernel, so a frame needs no bookkeeping launches.
struct Counters {
    unsigned long long touched_new; // this frame: low 32 bits |T_k| entries, high 32 bits new ones
    int32_t pool_used;   // allocated blocks
    int32_t frame_ok;    // 1 if the last frame was accepted
    uint32_t dirty_epoch;  // a block is dirty when its flag holds this value
    uint32_t mesh_epoch;   // epoch being meshed by the current extraction
    int32_t status;      // deferred error (MAP_ERR_CAPACITY) until read by the host
    int32_t frames;      // accepted frames
    unsigned long long mesh_tris;   // triangles of the last extraction
    unsigned long long mesh_blocks; // blocks of the last extraction
    unsigned long long last_updates;
    int32_t last_touched;  // |T_k| of the last accepted frame (labels read it)
    int32_t last_new;
    int32_t overflow;      // touched list overflow (cannot happen with the sizing rule)
    uint32_t extractions;  // extractions whose totals have been reported
    int32_t bits_gap;      // nonzero when a frame since the dirty set was last cleared did not
                           // mark the dirty bitmap (the next DIRTY extraction sweeps the slots)
    int32_t mesh_bits;     // the last extraction's candidates came from the dirty bitmap
};

// Same-address device atomics are serialised (about 12 ns apart on gfx950), so a value
// that every workgroup adds to is spread over kLeaves counters 128 bytes apart (a
// workgroup adds to leaf blockIdx % kLeaves) and summed by its single reader.
constexpr int kLeaves = 64;
constexpr int kLeafPad = 16;  // 64-bit words per leaf
struct Spread {
    unsigned long long v[kLeaves * kLeafPad];
};

// Hierarchical "last workgroup" ticket: a workgroup arrives at its leaf; the one that
// completes a leaf arrives at the root; the one that completes the root is last.
struct Ticket {
    unsigned long long leaf[kLeaves * kLeafPad];
    unsigned long long root[kLeafPad];
};

// Per-map synchronisation state (device, zero-initialised).
struct SyncState {
    Ticket tsdf;     // TSDF phase: the last workgroup closes the frame
    Spread updates;  // U_k being accumulated
    Spread votes;    // label votes since the last LiDAR frame
};

// One slot of the block hash, read with a single 16-byte load: the key (kEmpty: free),
// the block's pool slot, and the integration call that inserted it (~0 until its
// insertion completes).  Create fills every byte with 0xFF.
struct __align__(16) HashEntry {
    unsigned long long key;
    int32_t val;
    uint32_t frame;
};

// The whole entry in one 16-byte load (read field by field, the compiler would load the
// slot only after the key compared equal: a second dependent round trip).
__device__ __forceinline__ HashEntry hash_entry(const HashEntry *p)
{
    const uint4 v = *reinterpret_cast<const uint4 *>(p);
    HashEntry h;
    h.key = (unsigned long long)v.x | ((unsigned long long)v.y << 32);
    h.val = (int32_t)v.z;
    h.frame = v.w;
    return h;
}

// Block pool, hash and dirty set.
struct MapView {
    float2 *dw;               // [max_blocks][512] (D, W)
    uint8_t *fused;           // [max_blocks][512]
    uint16_t *counts;         // [max_blocks][L][512]
    int4 *coords;             // [max_blocks] block coordinates per slot; .w: epoch of the block's
                              // last dirty marking (dirty when it holds the current epoch)
    HashEntry *hash;          // [hmask + 1]
    uint16_t *mesh_cnt;       // [max_blocks] triangles of a block in the current extraction
    int32_t *mesh_nbr;        // [max_blocks][8] slots of b + e, e in {0,1}^3 (-1: absent), same
    unsigned long long *vmask;  // [max_blocks][16] per z slice: sign bits (D < 0), then observed
                                // bits (W > 0), bit y * 8 + x; kept by the TSDF pass
    float *grad;              // [max_blocks][3][512] unit distance gradient of the non-projective
                              // distance (x, y, z planes); null until that distance is enabled
    float *logpost;           // [max_blocks][L][512] class log-posteriors of Bayesian label fusion
                              // (largest 0); null until that fusion is enabled
    uint32_t *dbits;          // dirty bitmap in the meshing counting pass's order: slot
                              // s = w + j bits_grid is bit j % 32 of word w bits_wpw + j / 32,
                              // so counting workgroup w owns words [w bits_wpw, (w + 1) bits_wpw);
                              // a superset of the dirty set whenever ctr->bits_gap is 0 (kept
                              // only by frames that end with more than bits_from blocks)
    Counters *ctr;
    SyncState *sync;
    int32_t bits_from;        // frames mark, and DIRTY extractions read, the bitmap above this
                              // many allocated blocks (below it the slot sweep is one pass)
    int32_t bits_grid;        // counting grid the bitmap is laid out for
    int32_t bits_wpw;         // words per counting workgroup: ceil(ceil(max_blocks / grid) / 32)
    uint32_t hmask;
    int32_t n_classes;
    int32_t max_blocks;
    float nu, tau;
};

constexpr int kThreads = 256;      // threads of every workgroup of the library's kernels
constexpr int kMaxMeshGrid = 4096;  // workgroups of a meshing pass (and of a batched phase)

// A block with triangles, recorded by the counting pass of a per-map extraction for the
// emitting pass: its coordinates (x, y, z) and pool slot (w), and the slots of b + e,
// e in {0,1}^3 (-1 when absent).
struct __align__(16) MeshRec {
    int4 bc;
    int nb[8];
};

// Scratch of one extraction: per-workgroup triangle and block counts of the counting
// pass, and the output offsets of the emitting pass (per map of a batch: [grid][maps]).
// Per-map extractions also keep the counting pass's records: counting workgroup c writes
// its blocks with triangles, in its candidate order, to rec[c * rec_cap ...], and their
// number to wg_nz[c].
struct MeshScan {
    long long *wg_tris;
    int32_t *wg_blocks;
    long long *wg_off;
    MeshRec *rec;
    int32_t *wg_nz;
    int32_t rec_cap;
};

// An extraction's totals, written by the scan kernel straight into host-mapped pinned
// memory, so the host reads them after the stream wait without a copy launch.
struct MeshReport {
    unsigned long long tris;
    unsigned long long blocks;
    unsigned long long seq;  // the map's extraction number, stored last (release)
};

// Per-frame scratch: frame set (de-duplication of the frame's blocks) and touched list.
struct FrameView {
    unsigned long long *fkeys;  // [fmask + 1]
    unsigned long long *tk_key; // [tk_cap]
    int32_t *tk_slot;           // [tk_cap] pool slot (-1 until committed)
    int32_t *tk_rank;           // [tk_cap] rank among new blocks
    int32_t *tk_fslot;          // [tk_cap] frame-set slot (cleared at frame end)
    unsigned long long *band;   // [tk_cap][8] band bits (|psi| <= tau) per voxel
    float *rcopy;               // [rows * cols] the scan's range image, copied by the allocation
                                // launch (the TSDF launch, enqueued later, reads this copy)
    float4 *nimg;               // [rows * cols] non-projective distance: the scan's world-frame
                                // normals (xyz) and kept ranges (w, 0 where the point filter
                                // drops the return); null in projective mode
    uint32_t fmask;
    int32_t tk_cap;
};

// Sensor look-up tables (device), fp32 values each computed once in double.
struct LidarLUT {
    const float *ce, *se;   // ray elevation cos / sin, [rows]
    const float *cp, *sp;   // ray azimuth cos / sin, [cols]
    const float2 *bc;       // azimuth boundary between columns j-1 and j as (cos, sin), [cols]
    const float2 *br;       // elevation boundary j as (cos, sin), [rows + 1]
    int32_t rows, cols;
    float r_max;
    float cols_over_2pi;    // initial column guess scale
    float el_top;           // elevation of boundary 0 (initial row guess)
    float rows_over_fov;    // rows / (elevation of boundary 0 - elevation of boundary rows)
};

struct Pose {  // rows 0..2 of a row-major 4x4
    float m[12];
};

struct Camera {
    int32_t width, height;
    float fx, fy, cx, cy;
};

constexpr int kMaxCams = 8;
struct CameraSet {  // cameras fused by one launch, in call order
    int32_t n;
    Camera cam[kMaxCams];
    Pose T[kMaxCams];
    const uint8_t *img[kMaxCams];
};

struct MeshOut {
    float *pos;
    uint8_t *lab;
    long long *ekey;
    long long cap;
};

// ---------------------------------------------------------------------------------
// key packing and hashing (device + host)
// ---------------------------------------------------------------------------------
__host__ __device__ inline unsigned long long pack_key(int bx, int by, int bz)
{
    const long long bias = 1LL << 20;
    return ((unsigned long long)(bx + bias) << 42) | ((unsigned long long)(by + bias) << 21) |
           (unsigned long long)(bz + bias);
}

__host__ __device__ inline int3 unpack_key(unsigned long long k)
{
    const int bias = 1 << 20;
    return make_int3((int)((k >> 42) & 0x1FFFFF) - bias, (int)((k >> 21) & 0x1FFFFF) - bias,
                     (int)(k & 0x1FFFFF) - bias);
}

__host__ __device__ inline uint32_t hash_slot(unsigned long long k, uint32_t mask)
{
    k ^= k >> 33;
    k *= 0xff51afd7ed558ccdULL;
    k ^= k >> 33;
    k *= 0xc4ceb9fe1a85ec53ULL;
    k ^= k >> 33;
    return (uint32_t)k & mask;
}

__device__ inline int hash_find(const MapView &m, unsigned long long key)
{
    uint32_t i = hash_slot(key, m.hmask);
    for (uint32_t n = 0; n <= m.hmask; ++n) {
        const HashEntry h = hash_entry(&m.hash[i]);
        if (h.key == key) return h.val;
        if (h.key == kEmpty) return -1;
        i = (i + 1) & m.hmask;
    }
    return -1;
}

// ---------------------------------------------------------------------------------
// launch wrappers (defined in the kernel sources)
// ---------------------------------------------------------------------------------
// ---------------------------------------------------------------------------------
// batched steps: one launch per phase covers every map of the step
// ---------------------------------------------------------------------------------
constexpr int kMaxBatchMaps = 64;
constexpr int kBatchConcurrent = 4;   // batch schedule: each map's own kernels, maps over several streams
constexpr int kMaxBatchStreams = 16;  // streams of that schedule

struct BatchMap {  // one map's frame in a batched step (device array, refreshed per step)
    MapView v;
    FrameView f;
    LidarLUT lut;
    Pose T;
    const float *range;
    CameraSet cams;
    MeshOut out;
    int32_t tile0, tiles;  // this map's allocation tiles in the step's tile space
    uint32_t frame_id;     // this map's integration call number
};

// A frame's allocation outcome, read by every worker of its TSDF phase.
struct FrameState {
    int32_t n_list, n_new, used;
    uint32_t epoch;
    int32_t ok;
    int32_t bits;  // the frame marks the dirty bitmap (the pool ends above bits_from)
};

struct BatchCtl {  // device
    FrameState fs[kMaxBatchMaps];      // per-map frame state after allocation
    int32_t pre_t[kMaxBatchMaps + 1];  // prefix sums over maps: touched entries
    int32_t pre_l[kMaxBatchMaps + 1];  // label entries
    int32_t pre_p[kMaxBatchMaps + 1];  // mesh candidates (pool slots)
};

struct BatchSync {  // device, zero-initialised
    Ticket alloc;
    Ticket tsdf;
};

hipError_t launch_batch(BatchMap *maps, BatchCtl *ctl, BatchSync *sync, MeshScan scan, MeshReport *reports,
                        int n_maps, int total_tiles, int schedule, int grid, hipStream_t s);

hipError_t launch_init_pool(const MapView &m, hipStream_t s);
hipError_t launch_fill_u64(unsigned long long *p, size_t n, unsigned long long v, hipStream_t s);
// Distance of the TSDF update: the projective psi (the paper's Ours-Proj), or the
// non-projective distance of Eq. 4 with its normal image and point filter (Ours).
constexpr int kDistProjective = 0, kDistNonProjective = 1;
// Label fusion: vote counts (Eq. 6 with hard labels), the latest label (Ours-wo-Bay), or
// Eq. 6 on per-pixel class log-probabilities.
constexpr int kLabelCounts = 0, kLabelLatest = 1, kLabelBayes = 2;

hipError_t launch_alloc(const MapView &m, const FrameView &f, const LidarLUT &lut, const Pose &T,
                        const float *range, int dist_mode, float cos_inc, hipStream_t s);
// The TSDF launch, optionally fused with the label fusion of up to kMaxCams cameras
// (label_mode kLabelCounts or kLabelLatest; cams.n == 0: no labels).
hipError_t launch_tsdf(const MapView &m, const FrameView &f, const LidarLUT &lut, const Pose &T,
                       const float *range, uint32_t frame_id, int schedule, int grid, int dist_mode,
                       const CameraSet &cams, int label_mode, hipStream_t s);
hipError_t launch_labels(const MapView &m, const FrameView &f, const CameraSet &cams, int schedule, int grid,
                         int label_mode, hipStream_t s);
hipError_t launch_logprobs(const MapView &m, const FrameView &f, const Camera &cam, const Pose &T, const float *logp,
                           int grid, hipStream_t s);
// Workgroups of the meshing passes: the emitting pass's grid and the counting pass's,
// a multiple of it (each the device-resident grid of its kernel).
struct MeshGrid {
    int emit, count;
};
MeshGrid mesh_grid(int schedule);
MeshGrid batch_mesh_grid();
// Meshing is the counting pass, then the scan and the emitting pass (which may run on
// another stream once the counting pass is done).
hipError_t launch_mesh_count(const MapView &m, int mode, const MeshScan &scan, int schedule, MeshGrid grid,
                             bool allow_bits, hipStream_t s);
hipError_t launch_mesh_finish(const MapView &m, int mode, const MeshOut &out, const MeshScan &scan,
                              MeshReport *report, int schedule, MeshGrid grid, hipStream_t s);
hipError_t launch_labels_lidar(const MapView &m, const FrameView &f, const LidarLUT &lut, const Pose &T,
                               const uint8_t *img, int grid, int label_mode, hipStream_t s);
hipError_t launch_range_image(const LidarLUT &lut, const float *pts, int n, float F, float O,
                              unsigned long long *keys, float *depth, float *height, hipStream_t s);
// Uniform grid of a point cloud for capped nearest-neighbour queries (map-quality metrics):
// occupied cells in an open-addressing hash with their point counts and the offsets of
// their runs in pts (the cloud's points in cell order, point index bits in w).
struct CellGrid {
    unsigned long long *key;  // [mask + 1] packed cell coordinates (all ones: free)
    uint32_t *count;          // [mask + 1] points per cell (zeroed before the build)
    uint32_t *offset;         // [mask + 1] first point of the cell's run
    uint32_t *cursor;         // [mask + 1] fill cursor (zeroed before the build)
    uint32_t *slot_of;        // [n] cell slot of each point
    float4 *pts;              // [n] points in cell order
    uint32_t mask;
    double inv_h;             // 1 / cell edge
};
hipError_t launch_grid_build(CellGrid &g, const float *p, long long n, uint32_t *scan_tmp, hipStream_t s);
hipError_t launch_grid_query(const CellGrid &g, const float *q, long long n, double cap, double *dist, long long *nn,
                             hipStream_t s);
hipError_t launch_quality(const double *dM, long long nM, const double *dG, const long long *nnG, long long nG,
                          const uint8_t *labM, const uint8_t *labG, int L, double cap, double *partial, int nparts,
                          unsigned long long *conf, double *out, hipStream_t s);

hipError_t launch_query(const MapView &m, const float *pts, long long n, float *sdf, float *grad,
                        uint8_t *valid, hipStream_t s);
hipError_t launch_adjoint(const MapView &m, const float *xi, const float *pts, int B, long long N,
                          float *gpts, float *partial, int nchunk, hipStream_t s);
hipError_t launch_adjoint_reduce(const float *xi, const float *partial, int B, int nchunk,
                                 float *loss, float *gxi, hipStream_t s);

}  // namespace mc
