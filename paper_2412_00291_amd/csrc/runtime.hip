// Host runtime of mapcore: map object, argument checks, sensor look-up tables, scratch
// sizing and launch sequencing behind the C ABI declared in include/mapcore.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstddef>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <utility>
#include <vector>

#include "internal.h"
#include "mapcore.h"

using namespace mc;

struct map_s {
    map_params p{};
    MapView v{};
    FrameView f{};
    Counters *h_ctr = nullptr;  // pinned mirror for read-back
    MeshReport *h_report = nullptr;  // host-mapped, written by the extraction's scan kernel
    MeshReport *d_report = nullptr;  // the same memory as seen by the device
    hipEvent_t done = nullptr;       // recorded after an extraction (error detection)
    uint32_t n_extract = 0;          // extractions launched (the report's seq of the last one)
    hipStream_t last_stream = nullptr;
    bool has_scan = false;
    MeshScan scan{};        // extraction scratch, kMaxMeshGrid workgroups
    uint32_t frame_id = 0;  // integration calls so far (tags hash insertions)
    int sched[3] = {0, 0, 1};  // TSDF, labels, meshing: 0 workgroup / 1 wavefront per block
    int tsdf_grid = 1024;      // TSDF workgroups: six per compute unit of the map's device
    int64_t bits_user = -1;    // dirty-bitmap threshold set by the caller (< 0: the default)
    bool bits_relaid = false;  // the bitmap's layout changed since the last DIRTY extraction
    std::string err;
    // LiDAR look-up tables (device) and the model they were built for
    float *lut_buf = nullptr;
    size_t lut_floats = 0;
    LidarLUT lut{};
    int lut_rows = 0, lut_cols = 0;
    float lut_rmax = 0.0f;
    std::vector<float> lut_elev;
    // depth-buffer keys of the point-cloud preprocessing, one per pixel (all kNoPoint
    // between calls: the finishing pass resets what it reads)
    unsigned long long *rkeys = nullptr;
    int64_t rkeys_n = 0;
    bool rkeys_dirty = false;  // a failed call may have left keys set
    // distance and label-fusion modes (kDist*, kLabel*) and their buffers
    int dist_mode = kDistProjective;
    float cos_inc = 0.0f;      // point filter of the non-projective distance
    int64_t nimg_n = 0;        // pixels of the normal image (FrameView::nimg)
    int64_t rcopy_n = 0;       // pixels of the range copy (FrameView::rcopy)
    // The TSDF launch of the last LiDAR frame is enqueued by the map's next call: fused with
    // label fusion when that call fuses camera labels, on its own otherwise.  It reads only
    // the map's own buffers (the allocation launch copied the range image), so nothing of
    // the caller's has to outlive the call that enqueued the frame.
    struct {
        bool active = false;
        Pose T{};
        uint32_t fid = 0;
        hipStream_t s = nullptr;
    } pend;
    int label_mode = kLabelCounts;
    // adjoint partial sums
    float *partial = nullptr;
    size_t partial_floats = 0;
    // kernel timing: pending (kernel id, start, stop) event triples and a free list
    uint32_t prof_mask = 0;
    std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> prof_pending;
    std::vector<hipEvent_t> prof_free;
    double prof_ms[MAP_KERNEL_COUNT] = {};
    int64_t prof_n[MAP_KERNEL_COUNT] = {};
};

static std::string g_create_error;

// Dirty bitmap words per counting workgroup for a counting grid of G workgroups.
static int32_t bits_wpw(int64_t max_blocks, int G)
{
    return (int32_t)(((max_blocks + G - 1) / G + 31) / 32);
}

// The map's dirty-bitmap threshold and layout (MapView::bits_*): the caller's threshold,
// or the pool size that one round of the counting pass's slot sweep covers (one slot per
// thread of its grid); laid out for the counting grid of the current meshing schedule.
// A new layout leaves the current epoch's marks behind: the next DIRTY extraction sweeps.
static void set_bits(map_t *m)
{
    const int G = mesh_grid(m->sched[2]).count;
    const long long d = m->bits_user >= 0 ? m->bits_user : (long long)kThreads * G;
    m->v.bits_from = (int32_t)std::min<long long>(d, INT32_MAX);
    if (m->v.bits_grid != G) {
        m->v.bits_grid = G;
        m->v.bits_wpw = bits_wpw(m->p.max_blocks, G);
        m->bits_relaid = true;
    }
}

// Partial sums of map_sdf_pose_adjoint_noalloc: a file-scope device array (each device the
// library runs on holds its own copy until the process ends), so that call allocates
// nothing.  Its device address is looked up once per device, with that device current
// (map_create does it for its device), and kept here; host code uses only that address.
constexpr size_t kScratchFloats = (size_t)1 << 20;  // 4 MiB: B * ceil(N / 256) <= 131072 chunks
static __device__ __align__(256) float scratch[kScratchFloats];
constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mutex;
static float *g_scratch_ptr[kMaxDevices] = {};

// The device address of `scratch` on `device` (the current device), or null with *err set.
static float *scratch_on(int device, hipError_t *err)
{
    *err = hipSuccess;
    if (device < 0 || device >= kMaxDevices) {
        *err = hipErrorInvalidDevice;
        return nullptr;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[device]) {
        void *ptr = nullptr;
        *err = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (*err != hipSuccess) return nullptr;
        g_scratch_ptr[device] = static_cast<float *>(ptr);
    }
    return g_scratch_ptr[device];
}

static int fail(map_t *m, int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    if (m) m->err = buf;
    else g_create_error = buf;
    return code;
}

#define HIP_TRY(m, expr)                                                                          \
    do {                                                                                          \
        hipError_t e_ = (expr);                                                                   \
        if (e_ != hipSuccess)                                                                     \
            return fail((m), MAP_ERR_DEVICE, "%s: %s (%s:%d)", #expr, hipGetErrorString(e_), __FILE__, \
                        __LINE__);                                                                \
    } while (0)

// Wait for an extraction's report (written early in the emitting pass by its first
// workgroup; by the scan kernel in batched steps) by polling host-mapped memory, so the
// call returns while the triangles are still being emitted on the stream.  Every 64 polls the event recorded
// after the extraction is queried: a device error ends the wait, and so does the
// extraction's completion without the expected report (hipErrorUnknown).
static hipError_t wait_report(const MeshReport *r, uint32_t seq, hipEvent_t done)
{
    for (unsigned i = 1;; ++i) {
        if (__atomic_load_n(&r->seq, __ATOMIC_ACQUIRE) == seq) return hipSuccess;
        if (i % 64) continue;
        const hipError_t q = hipEventQuery(done);
        if (q == hipErrorNotReady) continue;
        if (q != hipSuccess) return q;
        return __atomic_load_n(&r->seq, __ATOMIC_ACQUIRE) == seq ? hipSuccess : hipErrorUnknown;
    }
}

static uint64_t next_pow2(uint64_t x)
{
    uint64_t p = 1;
    while (p < x) p <<= 1;
    return p;
}

static void free_all(map_t *m)
{
    for (auto &p : m->prof_pending) {
        (void)hipEventDestroy(p.second.first);
        (void)hipEventDestroy(p.second.second);
    }
    for (hipEvent_t e : m->prof_free) (void)hipEventDestroy(e);
    m->prof_pending.clear();
    m->prof_free.clear();
    void *ptrs[] = {m->v.dw, m->v.fused, m->v.counts, m->v.coords, m->v.hash,
                    m->v.mesh_cnt, m->v.mesh_nbr, m->v.vmask, m->v.dbits, m->v.ctr, m->v.sync, m->f.fkeys, m->f.tk_key, m->f.tk_slot, m->f.tk_rank,
                    m->f.tk_fslot, m->f.band, m->f.nimg, m->f.rcopy, m->v.grad, m->v.logpost, m->lut_buf, m->partial,
                    m->scan.wg_tris, m->scan.wg_blocks, m->scan.wg_off, m->scan.rec, m->scan.wg_nz, m->rkeys};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    if (m->h_ctr) (void)hipHostFree(m->h_ctr);
    if (m->h_report) (void)hipHostFree(m->h_report);
    if (m->done) (void)hipEventDestroy(m->done);
}

// rigid transform check: finite, last row (0,0,0,1), orthonormal rotation to 1e-5, det > 0
static bool pose_ok(const float *T)
{
    for (int i = 0; i < 16; ++i)
        if (!std::isfinite(T[i])) return false;
    if (T[12] != 0.0f || T[13] != 0.0f || T[14] != 0.0f || T[15] != 1.0f) return false;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double s = 0.0;
            for (int k = 0; k < 3; ++k) s += (double)T[4 * k + i] * (double)T[4 * k + j];
            if (std::fabs(s - (i == j ? 1.0 : 0.0)) > 1e-5) return false;
        }
    double det = (double)T[0] * ((double)T[5] * T[10] - (double)T[6] * T[9]) -
                 (double)T[1] * ((double)T[4] * T[10] - (double)T[6] * T[8]) +
                 (double)T[2] * ((double)T[4] * T[9] - (double)T[5] * T[8]);
    return det > 0.0;
}

static hipEvent_t take_event(map_t *m)
{
    if (!m->prof_free.empty()) {
        hipEvent_t e = m->prof_free.back();
        m->prof_free.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Launch through `fn`, bracketed by events on the same stream when kernel `kid` is timed.
template <class F>
static hipError_t timed(map_t *m, int kid, hipStream_t s, F fn)
{
    if (!((m->prof_mask >> kid) & 1u)) return fn();
    hipEvent_t a = take_event(m), b = take_event(m);
    if (!a || !b) return hipErrorOutOfMemory;
    hipError_t e = hipEventRecord(a, s);
    if (e != hipSuccess) return e;
    e = fn();
    if (e != hipSuccess) return e;
    e = hipEventRecord(b, s);
    if (e != hipSuccess) return e;
    m->prof_pending.push_back({kid, {a, b}});
    return hipSuccess;
}

static int flush_pending(map_t *m);

extern "C" int map_profile(map_t *m, uint32_t mask)
{
    if (!m) return MAP_ERR_INVALID_ARG;
    {
        const int rc = flush_pending(m);  // a pending launch is timed under the mask it was enqueued with
        if (rc) return rc;
    }
    m->prof_mask = mask & ((1u << MAP_KERNEL_COUNT) - 1);
    return MAP_OK;
}

extern "C" int map_profile_read(map_t *m, double *total_ms, int64_t *launches)
{
    if (!m) return MAP_ERR_INVALID_ARG;
    {
        const int rc = flush_pending(m);
        if (rc) return rc;
    }
    HIP_TRY(m, hipSetDevice(m->p.device));
    for (auto &p : m->prof_pending) {
        HIP_TRY(m, hipEventSynchronize(p.second.second));
        float ms = 0.0f;
        HIP_TRY(m, hipEventElapsedTime(&ms, p.second.first, p.second.second));
        m->prof_ms[p.first] += ms;
        m->prof_n[p.first] += 1;
        m->prof_free.push_back(p.second.first);
        m->prof_free.push_back(p.second.second);
    }
    m->prof_pending.clear();
    for (int k = 0; k < MAP_KERNEL_COUNT; ++k) {
        if (total_ms) total_ms[k] = m->prof_ms[k];
        if (launches) launches[k] = m->prof_n[k];
        m->prof_ms[k] = 0.0;
        m->prof_n[k] = 0;
    }
    return MAP_OK;
}

static Pose to_pose(const float *T)
{
    Pose P;
    for (int i = 0; i < 12; ++i) P.m[i] = T[i];
    return P;
}

extern "C" int map_create(const map_params *params, void *stream, map_t **out)
{
    if (!params || !out) return fail(nullptr, MAP_ERR_INVALID_ARG, "map_create: NULL argument");
    *out = nullptr;
    const map_params &p = *params;
    if (!(p.voxel_size > 0.0f) || !std::isfinite(p.voxel_size) || !(p.truncation > 0.0f) ||
        !std::isfinite(p.truncation) || p.truncation > 64.0f * p.voxel_size)
        return fail(nullptr, MAP_ERR_INVALID_ARG, "map_create: need voxel_size > 0 and 0 < truncation <= 64 voxel_size");
    if (p.n_classes < 1 || p.n_classes > 254)
        return fail(nullptr, MAP_ERR_INVALID_ARG, "map_create: n_classes must be in [1, 254]");
    if (p.max_blocks < 1 || p.max_blocks > (int64_t)1 << 30)
        return fail(nullptr, MAP_ERR_INVALID_ARG, "map_create: max_blocks must be in [1, 2^30]");
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || p.device < 0 || p.device >= ndev)
        return fail(nullptr, MAP_ERR_INVALID_ARG, "map_create: device %d not available", p.device);
    if (hipSetDevice(p.device) != hipSuccess)
        return fail(nullptr, MAP_ERR_DEVICE, "map_create: hipSetDevice failed");

    {  // set-up of the allocation-free adjoint's scratch on this device (once per device)
        hipError_t se;
        if (!scratch_on(p.device, &se))
            return fail(nullptr, MAP_ERR_DEVICE, "map_create: scratch address: %s", hipGetErrorString(se));
    }
    map_t *m = new map_s();
    m->p = p;
    // Six TSDF workgroups per compute unit: measured on a street frame (64 x 2048 scan,
    // 0.1 m voxels), four and seven per unit take 7% and 17% longer.
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, p.device) == hipSuccess && cus > 0)
        m->tsdf_grid = 6 * cus;
    hipStream_t s = (hipStream_t)stream;
    m->last_stream = s;
    const size_t nb = (size_t)p.max_blocks;
    const uint64_t hcap = next_pow2(std::max<uint64_t>(2 * nb, 1024));
    MapView &v = m->v;
    v.hmask = (uint32_t)(hcap - 1);
    v.n_classes = p.n_classes;
    v.max_blocks = (int32_t)p.max_blocks;
    v.nu = p.voxel_size;
    v.tau = p.truncation;
    auto cleanup = [&](int code) {
        int rc = fail(nullptr, code, "map_create: %s", m->err.c_str());
        free_all(m);
        delete m;
        return rc;
    };
#define CREATE_TRY(expr)                                                                  \
    do {                                                                                  \
        hipError_t e_ = (expr);                                                           \
        if (e_ != hipSuccess) {                                                           \
            m->err = std::string(#expr) + ": " + hipGetErrorString(e_);                   \
            return cleanup(MAP_ERR_DEVICE);                                               \
        }                                                                                 \
    } while (0)
    CREATE_TRY(hipMalloc(&v.dw, nb * kBlockVoxels * sizeof(float2)));
    CREATE_TRY(hipMalloc(&v.fused, nb * kBlockVoxels));
    CREATE_TRY(hipMalloc(&v.counts, nb * (size_t)p.n_classes * kBlockVoxels * sizeof(uint16_t)));
    CREATE_TRY(hipMalloc(&v.coords, nb * sizeof(int4)));
    CREATE_TRY(hipMalloc(&v.hash, hcap * sizeof(HashEntry)));
    CREATE_TRY(hipMalloc(&v.mesh_cnt, nb * sizeof(uint16_t)));
    CREATE_TRY(hipMalloc(&v.mesh_nbr, nb * 8 * sizeof(int32_t)));
    CREATE_TRY(hipMalloc(&v.vmask, nb * 16 * sizeof(unsigned long long)));
    // the dirty bitmap, sized for the layout of either meshing schedule's counting grid
    size_t bit_words = 0;
    for (int sc = 0; sc < 2; ++sc) {
        const int G = mesh_grid(sc).count;
        bit_words = std::max(bit_words, (size_t)G * bits_wpw(p.max_blocks, G));
    }
    CREATE_TRY(hipMalloc(&v.dbits, bit_words * sizeof(uint32_t)));
    CREATE_TRY(hipMalloc(&v.ctr, sizeof(Counters)));
    CREATE_TRY(hipMalloc(&v.sync, sizeof(SyncState)));
    CREATE_TRY(hipMalloc(&m->scan.wg_tris, kMaxMeshGrid * sizeof(long long)));
    CREATE_TRY(hipMalloc(&m->scan.wg_blocks, kMaxMeshGrid * sizeof(int32_t)));
    CREATE_TRY(hipMalloc(&m->scan.wg_off, kMaxMeshGrid * sizeof(long long)));
    // records of the counting pass: a segment of ceil(max_blocks / G) + 256 per counting
    // workgroup, for any grid G <= kMaxMeshGrid
    CREATE_TRY(hipMalloc(&m->scan.rec, (nb + 257 * (size_t)kMaxMeshGrid) * sizeof(MeshRec)));
    CREATE_TRY(hipMalloc(&m->scan.wg_nz, kMaxMeshGrid * sizeof(int32_t)));
    CREATE_TRY(hipHostMalloc((void **)&m->h_ctr, sizeof(Counters), hipHostMallocDefault));
    CREATE_TRY(hipHostMalloc((void **)&m->h_report, sizeof(MeshReport), hipHostMallocMapped | hipHostMallocCoherent));
    std::memset(m->h_report, 0, sizeof(MeshReport));
    CREATE_TRY(hipHostGetDevicePointer((void **)&m->d_report, m->h_report, 0));
    CREATE_TRY(hipEventCreateWithFlags(&m->done, hipEventDisableTiming));
    CREATE_TRY(hipMemsetAsync(v.dw, 0, nb * kBlockVoxels * sizeof(float2), s));
    CREATE_TRY(hipMemsetAsync(v.counts, 0, nb * (size_t)p.n_classes * kBlockVoxels * sizeof(uint16_t), s));
    CREATE_TRY(hipMemsetAsync(v.coords, 0, nb * sizeof(int4), s));
    CREATE_TRY(hipMemsetAsync(v.vmask, 0, nb * 16 * sizeof(unsigned long long), s));
    CREATE_TRY(hipMemsetAsync(v.dbits, 0, bit_words * sizeof(uint32_t), s));
    set_bits(m);
    m->bits_relaid = false;  // no frame yet
    CREATE_TRY(hipMemsetAsync(v.sync, 0, sizeof(SyncState), s));
    CREATE_TRY(hipMemsetAsync(v.hash, 0xFF, hcap * sizeof(HashEntry), s));  // free keys, no insertion
    CREATE_TRY(launch_init_pool(v, s));
    std::memset(m->h_ctr, 0, sizeof(Counters));
    m->h_ctr->dirty_epoch = 1;
    CREATE_TRY(hipMemcpyAsync(v.ctr, m->h_ctr, sizeof(Counters), hipMemcpyHostToDevice, s));
    CREATE_TRY(hipStreamSynchronize(s));
#undef CREATE_TRY
    *out = m;
    return MAP_OK;
}

extern "C" void map_destroy(map_t *m)
{
    if (!m) return;
    (void)hipSetDevice(m->p.device);
    (void)hipDeviceSynchronize();
    free_all(m);
    delete m;
}

extern "C" const char *map_last_error(const map_t *m)
{
    return m ? m->err.c_str() : g_create_error.c_str();
}

// Build (or reuse) the look-up tables of a LiDAR model.  Values are computed in double
// and rounded once to fp32: ray directions from cos / sin of the row elevation and of
// the column azimuth pi - c 2pi/C; column boundaries at pi - (c - 1/2) 2pi/C; row
// boundaries halfway between neighbouring elevations, the outer ones half a spacing
// beyond the first and last rows.
static int ensure_lut(map_t *m, const lidar_model *L, hipStream_t s)
{
    const int R = L->rows, C = L->cols;
    if (m->lut_buf && m->lut_rows == R && m->lut_cols == C && m->lut_rmax == L->r_max &&
        std::memcmp(m->lut_elev.data(), L->elev_rad, R * sizeof(float)) == 0)
        return MAP_OK;
    for (int k = 0; k < R; ++k)
        if (!std::isfinite(L->elev_rad[k])) return fail(m, MAP_ERR_INVALID_ARG, "lidar: non-finite elevation");
    for (int k = 1; k < R; ++k)
        if (!(L->elev_rad[k] < L->elev_rad[k - 1]))
            return fail(m, MAP_ERR_INVALID_ARG, "lidar: elevations must strictly decrease (top row first)");
    const double e0 = L->elev_rad[0], e1 = L->elev_rad[1], en = L->elev_rad[R - 1], en1 = L->elev_rad[R - 2];
    const double top = e0 + 0.5 * (e0 - e1), bot = en - 0.5 * (en1 - en);
    if (!(top < M_PI / 2) || !(bot > -M_PI / 2))
        return fail(m, MAP_ERR_INVALID_ARG, "lidar: vertical field of view must stay within +-90 degrees");
    const size_t nfl = 2 * (size_t)R + 4 * (size_t)C + 2 * ((size_t)R + 1);
    std::vector<float> h(nfl);
    // ce[R] se[R] cp[C] sp[C], then (cos, sin) pairs: bc[C], br[R + 1] (8-byte aligned)
    float *ce = h.data(), *se = ce + R, *cp = se + R, *sp = cp + C, *bc = sp + C, *br = bc + 2 * C;
    for (int k = 0; k < R; ++k) {
        ce[k] = (float)std::cos((double)L->elev_rad[k]);
        se[k] = (float)std::sin((double)L->elev_rad[k]);
    }
    const double dphi = 2.0 * M_PI / (double)C;
    for (int c = 0; c < C; ++c) {
        const double phi = M_PI - (double)c * dphi;
        cp[c] = (float)std::cos(phi);
        sp[c] = (float)std::sin(phi);
        const double pb = M_PI - ((double)c - 0.5) * dphi;
        bc[2 * c] = (float)std::cos(pb);
        bc[2 * c + 1] = (float)std::sin(pb);
    }
    for (int j = 0; j <= R; ++j) {
        double eb = j == 0 ? top : (j == R ? bot : 0.5 * ((double)L->elev_rad[j - 1] + (double)L->elev_rad[j]));
        br[2 * j] = (float)std::cos(eb);
        br[2 * j + 1] = (float)std::sin(eb);
    }
    // the previous frame may still read the old tables
    HIP_TRY(m, hipStreamSynchronize(s));
    if (nfl > m->lut_floats) {
        if (m->lut_buf) HIP_TRY(m, hipFree(m->lut_buf));
        m->lut_buf = nullptr;
        HIP_TRY(m, hipMalloc(&m->lut_buf, nfl * sizeof(float)));
        m->lut_floats = nfl;
    }
    HIP_TRY(m, hipMemcpy(m->lut_buf, h.data(), nfl * sizeof(float), hipMemcpyHostToDevice));
    float *d = m->lut_buf;
    LidarLUT &lut = m->lut;
    lut.ce = d;
    lut.se = d + R;
    lut.cp = d + 2 * R;
    lut.sp = lut.cp + C;
    lut.bc = reinterpret_cast<const float2 *>(lut.sp + C);
    lut.br = lut.bc + C;
    lut.rows = R;
    lut.cols = C;
    lut.r_max = L->r_max;
    lut.cols_over_2pi = (float)((double)C / (2.0 * M_PI));
    lut.el_top = (float)top;
    lut.rows_over_fov = (float)((double)R / (top - bot));
    m->lut_rows = R;
    m->lut_cols = C;
    m->lut_rmax = L->r_max;
    m->lut_elev.assign(L->elev_rad, L->elev_rad + R);
    return MAP_OK;
}

// Touched-list capacity for a model: every return meets at most 1 + 3 (floor(L / 8) + 1)
// blocks along a band of L = 2 tau / nu voxels (one per boundary crossing per axis).
static int ensure_frame_scratch(map_t *m, const lidar_model *L, hipStream_t s)
{
    const double band_vox = 2.0 * (double)m->p.truncation / (double)m->p.voxel_size;
    const int64_t per_ray = 1 + 3 * ((int64_t)std::floor(band_vox / 8.0) + 2);
    const int64_t need = (int64_t)L->rows * L->cols * per_ray;
    if (need > (int64_t)1 << 30) return fail(m, MAP_ERR_INVALID_ARG, "lidar: image too large");
    if (m->dist_mode == kDistNonProjective && (int64_t)L->rows * L->cols > m->nimg_n) {
        HIP_TRY(m, hipStreamSynchronize(s));
        if (m->f.nimg) HIP_TRY(m, hipFree(m->f.nimg));
        m->f.nimg = nullptr;
        m->nimg_n = 0;
        HIP_TRY(m, hipMalloc(&m->f.nimg, (size_t)L->rows * L->cols * sizeof(float4)));
        m->nimg_n = (int64_t)L->rows * L->cols;
    }
    if ((int64_t)L->rows * L->cols > m->rcopy_n) {
        HIP_TRY(m, hipStreamSynchronize(s));
        if (m->f.rcopy) HIP_TRY(m, hipFree(m->f.rcopy));
        m->f.rcopy = nullptr;
        m->rcopy_n = 0;
        HIP_TRY(m, hipMalloc(&m->f.rcopy, (size_t)L->rows * L->cols * sizeof(float)));
        m->rcopy_n = (int64_t)L->rows * L->cols;
    }
    if (m->f.tk_cap >= need) return MAP_OK;
    HIP_TRY(m, hipStreamSynchronize(s));
    FrameView &f = m->f;
    void *old[] = {f.fkeys, f.tk_key, f.tk_slot, f.tk_rank, f.tk_fslot, f.band};
    for (void *p : old)
        if (p) HIP_TRY(m, hipFree(p));
    float4 *nimg = f.nimg;  // kept (sized separately)
    float *rcopy = f.rcopy;
    f = FrameView{};
    f.nimg = nimg;
    f.rcopy = rcopy;
    const uint64_t fcap = next_pow2((uint64_t)(2 * need));
    HIP_TRY(m, hipMalloc(&f.fkeys, fcap * sizeof(unsigned long long)));
    HIP_TRY(m, hipMalloc(&f.tk_key, need * sizeof(unsigned long long)));
    HIP_TRY(m, hipMalloc(&f.tk_slot, need * sizeof(int32_t)));
    HIP_TRY(m, hipMalloc(&f.tk_rank, need * sizeof(int32_t)));
    HIP_TRY(m, hipMalloc(&f.tk_fslot, need * sizeof(int32_t)));
    HIP_TRY(m, hipMalloc(&f.band, need * 8 * sizeof(unsigned long long)));
    HIP_TRY(m, launch_fill_u64(f.fkeys, fcap, kEmpty, s));
    f.fmask = (uint32_t)(fcap - 1);
    f.tk_cap = (int32_t)need;
    return MAP_OK;
}

static int grid_for(int64_t items, int per_block, int cap)
{
    int64_t g = (items + per_block - 1) / per_block;
    if (g < 1) g = 1;
    return (int)(g < cap ? g : cap);
}

// Enqueue the last frame's TSDF launch (fused with the label fusion of the cameras in cs when
// cs.n > 0), on the stream of the frame's allocation launch.
static int launch_pending(map_t *m, const CameraSet &cs)
{
    if (!m->pend.active) return MAP_OK;
    m->pend.active = false;
    HIP_TRY(m, hipSetDevice(m->p.device));
    const hipStream_t s = m->pend.s;
    HIP_TRY(m, timed(m, cs.n > 0 ? MAP_K_TSDF_LABELS : MAP_K_TSDF, s, [&] {
        return launch_tsdf(m->v, m->f, m->lut, m->pend.T, m->f.rcopy, m->pend.fid, m->sched[0],
                           grid_for(m->f.tk_cap, 1, m->tsdf_grid), m->dist_mode, cs, m->label_mode, s);
    }));
    m->last_stream = s;
    return MAP_OK;
}

static int flush_pending(map_t *m) { return launch_pending(m, CameraSet{}); }

#define FLUSH_PENDING(m)                        \
    do {                                        \
        const int rc_ = flush_pending(m);       \
        if (rc_) return rc_;                    \
    } while (0)

extern "C" int map_integrate_lidar(map_t *m, const lidar_model *L, const float *range_dev, const float T_wl[16],
                                   void *stream)
{
    if (!m) return MAP_ERR_INVALID_ARG;
    if (!L || !range_dev || !T_wl || !L->elev_rad) return fail(m, MAP_ERR_INVALID_ARG, "integrate_lidar: NULL argument");
    if (L->rows < 2 || L->cols < 8) return fail(m, MAP_ERR_INVALID_ARG, "integrate_lidar: need rows >= 2, cols >= 8");
    if (!(L->r_max > 0.0f) || !std::isfinite(L->r_max))
        return fail(m, MAP_ERR_INVALID_ARG, "integrate_lidar: r_max must be positive and finite");
    if (!pose_ok(T_wl)) return fail(m, MAP_ERR_INVALID_ARG, "integrate_lidar: pose is not a rigid transform");
    const double lim = (double)m->p.voxel_size * kDomainVoxels;
    for (int i = 0; i < 3; ++i)
        if (std::fabs((double)T_wl[4 * i + 3]) + (double)L->r_max + (double)m->p.truncation >= lim)
            return fail(m, MAP_ERR_INVALID_ARG, "integrate_lidar: scan reaches outside the map domain");
    hipStream_t s = (hipStream_t)stream;
    int rc = flush_pending(m);
    if (rc) return rc;
    HIP_TRY(m, hipSetDevice(m->p.device));
    rc = ensure_lut(m, L, s);
    if (rc) return rc;
    rc = ensure_frame_scratch(m, L, s);
    if (rc) return rc;
    const Pose T = to_pose(T_wl);
    HIP_TRY(m, timed(m, MAP_K_ALLOC, s, [&] {
        return launch_alloc(m->v, m->f, m->lut, T, range_dev, m->dist_mode, m->cos_inc, s);
    }));
    m->pend.active = true;
    m->pend.T = T;
    m->pend.fid = m->frame_id++;
    m->pend.s = s;
    m->last_stream = s;
    m->has_scan = true;
    return MAP_OK;
}

static bool camera_ok(const camera_model *cam)
{
    return cam->width >= 1 && cam->height >= 1 && std::isfinite(cam->fx) && std::isfinite(cam->fy) &&
           std::isfinite(cam->cx) && std::isfinite(cam->cy) && cam->fx != 0.0f && cam->fy != 0.0f;
}

extern "C" int map_integrate_labels_multi(map_t *m, int32_t n, const camera_model *cams,
                                          const uint8_t *const *labels_dev, const float *T_wc, void *stream)
{
    if (!m) return MAP_ERR_INVALID_ARG;
    if (n < 1 || !cams || !labels_dev || !T_wc) return fail(m, MAP_ERR_INVALID_ARG, "integrate_labels: bad arguments");
    for (int i = 0; i < n; ++i) {
        if (!labels_dev[i]) return fail(m, MAP_ERR_INVALID_ARG, "integrate_labels: NULL label image %d", i);
        if (!camera_ok(&cams[i])) return fail(m, MAP_ERR_INVALID_ARG, "integrate_labels: bad camera model %d", i);
        if (!pose_ok(T_wc + 16 * i)) return fail(m, MAP_ERR_INVALID_ARG, "integrate_labels: pose %d is not rigid", i);
    }
    if (m->label_mode == kLabelBayes)
        return fail(m, MAP_ERR_INVALID_ARG, "integrate_labels: the map fuses log-probability images");
    if (!m->has_scan) return fail(m, MAP_ERR_NO_SCAN, "integrate_labels: no LiDAR frame integrated yet");
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(m, hipSetDevice(m->p.device));
    // a frame whose TSDF launch is still to come takes the first cameras into that launch
    const bool fuse = m->pend.active && m->pend.s == s;
    if (!fuse) {
        const int rc = flush_pending(m);
        if (rc) return rc;
    }
    for (int i0 = 0; i0 < n; i0 += kMaxCams) {
        CameraSet cs{};
        cs.n = std::min(kMaxCams, n - i0);
        for (int j = 0; j < cs.n; ++j) {
            const camera_model &c = cams[i0 + j];
            cs.cam[j] = Camera{c.width, c.height, c.fx, c.fy, c.cx, c.cy};
            cs.T[j] = to_pose(T_wc + 16 * (i0 + j));
            cs.img[j] = labels_dev[i0 + j];
        }
        if (i0 == 0 && fuse) {
            const int rc = launch_pending(m, cs);
            if (rc) return rc;
            continue;
        }
        HIP_TRY(m, timed(m, MAP_K_LABELS, s, [&] {
            return launch_labels(m->v, m->f, cs, m->sched[1], grid_for(m->f.tk_cap, 1, 2048), m->label_mode, s);
        }));
    }
    m->last_stream = s;
    return MAP_OK;
}

extern "C" int map_integrate_labels_lidar(map_t *m, const lidar_model *L, const uint8_t *labels_dev,
                                          const float T_wl[16], void *stream)
{
    if (!m) return MAP_ERR_INVALID_ARG;
    FLUSH_PENDING(m);
    if (!L || !labels_dev || !T_wl || !L->elev_rad)
        return fail(m, MAP_ERR_INVALID_ARG, "integrate_labels_lidar: NULL argument");
    if (L->rows < 2 || L->cols < 8) return fail(m, MAP_ERR_INVALID_ARG, "integrate_labels_lidar: need rows >= 2, cols >= 8");
    if (!(L->r_max > 0.0f) || !std::isfinite(L->r_max))
        return fail(m, MAP_ERR_INVALID_ARG, "integrate_labels_lidar: r_max must be positive and finite");
    if (!pose_ok(T_wl)) return fail(m, MAP_ERR_INVALID_ARG, "integrate_labels_lidar: pose is not a rigid transform");
    if (m->label_mode == kLabelBayes)
        return fail(m, MAP_ERR_INVALID_ARG, "integrate_labels_lidar: the map fuses log-probability images");
    if (!m->has_scan) return fail(m, MAP_ERR_NO_SCAN, "integrate_labels_lidar: no LiDAR frame integrated yet");
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(m, hipSetDevice(m->p.device));
    const int rc = ensure_lut(m, L, s);
    if (rc) return rc;
    const Pose T = to_pose(T_wl);
    HIP_TRY(m, timed(m, MAP_K_LABELS, s, [&] {
        return launch_labels_lidar(m->v, m->f, m->lut, T, labels_dev, grid_for(m->f.tk_cap, 1, 2048), m->label_mode,
                                   s);
    }));
    m->last_stream = s;
    return MAP_OK;
}

extern "C" int map_set_distance(map_t *m, int32_t mode, float max_incidence)
{
    if (!m) return MAP_ERR_INVALID_ARG;
    FLUSH_PENDING(m);
    if ((mode != MAP_DIST_PROJECTIVE && mode != MAP_DIST_NONPROJECTIVE) || !std::isfinite(max_incidence) ||
        max_incidence < 0.0f)
        return fail(m, MAP_ERR_INVALID_ARG, "set_distance: mode 0 or 1 and a finite max_incidence >= 0");
    HIP_TRY(m, hipSetDevice(m->p.device));
    if (mode == MAP_DIST_NONPROJECTIVE && !m->v.grad) {
        const size_t bytes = (size_t)m->p.max_blocks * 3 * kBlockVoxels * sizeof(float);
        HIP_TRY(m, hipStreamSynchronize(m->last_stream));
        HIP_TRY(m, hipMalloc(&m->v.grad, bytes));
        HIP_TRY(m, hipMemset(m->v.grad, 0, bytes));
    }
    m->dist_mode = mode;
    m->cos_inc = (float)std::cos((double)max_incidence);
    return MAP_OK;
}

extern "C" int map_set_label_fusion(map_t *m, int32_t mode)
{
    if (!m) return MAP_ERR_INVALID_ARG;
    FLUSH_PENDING(m);
    if (mode != MAP_LABELS_COUNTS && mode != MAP_LABELS_LATEST && mode != MAP_LABELS_BAYES)
        return fail(m, MAP_ERR_INVALID_ARG, "set_label_fusion: mode 0, 1 or 2");
    HIP_TRY(m, hipSetDevice(m->p.device));
    if (mode == MAP_LABELS_BAYES && !m->v.logpost) {
        const size_t bytes = (size_t)m->p.max_blocks * m->p.n_classes * kBlockVoxels * sizeof(float);
        HIP_TRY(m, hipStreamSynchronize(m->last_stream));
        HIP_TRY(m, hipMalloc(&m->v.logpost, bytes));
        HIP_TRY(m, hipMemset(m->v.logpost, 0, bytes));
    }
    m->label_mode = mode;
    return MAP_OK;
}

extern "C" int map_integrate_logprobs(map_t *m, const camera_model *cam, const float *logp_dev, const float T_wc[16],
                                      void *stream)
{
    if (!m) return MAP_ERR_INVALID_ARG;
    FLUSH_PENDING(m);
    if (!cam || !logp_dev || !T_wc) return fail(m, MAP_ERR_INVALID_ARG, "integrate_logprobs: NULL argument");
    if (!camera_ok(cam)) return fail(m, MAP_ERR_INVALID_ARG, "integrate_logprobs: bad camera model");
    if (!pose_ok(T_wc)) return fail(m, MAP_ERR_INVALID_ARG, "integrate_logprobs: pose is not a rigid transform");
    if (m->label_mode != kLabelBayes)
        return fail(m, MAP_ERR_INVALID_ARG, "integrate_logprobs: the map's label fusion is not Bayesian (mode 2)");
    if (!m->has_scan) return fail(m, MAP_ERR_NO_SCAN, "integrate_logprobs: no LiDAR frame integrated yet");
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(m, hipSetDevice(m->p.device));
    const Camera c{cam->width, cam->height, cam->fx, cam->fy, cam->cx, cam->cy};
    const Pose T = to_pose(T_wc);
    HIP_TRY(m, timed(m, MAP_K_LABELS, s, [&] {
        return launch_logprobs(m->v, m->f, c, T, logp_dev, grid_for(m->f.tk_cap, 1, 2048), s);
    }));
    m->last_stream = s;
    return MAP_OK;
}

extern "C" int map_integrate_labels(map_t *m, const camera_model *cam, const uint8_t *labels_dev,
                                    const float T_wc[16], void *stream)
{
    if (!m) return MAP_ERR_INVALID_ARG;
    if (!cam || !labels_dev || !T_wc) return fail(m, MAP_ERR_INVALID_ARG, "integrate_labels: NULL argument");
    return map_integrate_labels_multi(m, 1, cam, &labels_dev, T_wc, stream);
}

extern "C" int map_extract_mesh(map_t *m, int mode, float *pos_dev, uint8_t *lab_dev, int64_t *edge_keys_dev,
                                int64_t cap_tris, int64_t *n_tris, void *stream)
{
    if (!m) return MAP_ERR_INVALID_ARG;
    FLUSH_PENDING(m);
    if (!n_tris || cap_tris < 0 || (mode != MAP_MESH_DIRTY && mode != MAP_MESH_ALL))
        return fail(m, MAP_ERR_INVALID_ARG, "extract_mesh: bad mode, capacity or n_tris");
    if (cap_tris > 0 && (!pos_dev || !lab_dev)) return fail(m, MAP_ERR_INVALID_ARG, "extract_mesh: NULL output");
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(m, hipSetDevice(m->p.device));
    MeshOut out{pos_dev, lab_dev, (long long *)edge_keys_dev, (long long)cap_tris};
    const MeshGrid grid = mesh_grid(m->sched[2]);
    m->scan.rec_cap = (int32_t)((m->p.max_blocks + grid.count - 1) / grid.count + 256);
    HIP_TRY(m, timed(m, MAP_K_MESH, s, [&] {
        hipError_t e = launch_mesh_count(m->v, mode, m->scan, m->sched[2], grid, !m->bits_relaid, s);
        return e != hipSuccess ? e : launch_mesh_finish(m->v, mode, out, m->scan, m->d_report, m->sched[2], grid, s);
    }));
    if (mode == MAP_MESH_DIRTY) m->bits_relaid = false;  // it swept; one that did not fit leaves the gap flag
    HIP_TRY(m, hipEventRecord(m->done, s));
    m->last_stream = s;
    const uint32_t seq = ++m->n_extract;
    const hipError_t we = wait_report(m->h_report, seq, m->done);
    if (we != hipSuccess) {
        m->n_extract = (uint32_t)__atomic_load_n(&m->h_report->seq, __ATOMIC_ACQUIRE);
        return fail(m, MAP_ERR_DEVICE, "extract_mesh: %s", hipGetErrorString(we));
    }
    const int64_t n = (int64_t)__atomic_load_n(&m->h_report->tris, __ATOMIC_ACQUIRE);
    *n_tris = n;
    if (n > cap_tris)
        return fail(m, MAP_ERR_BUFFER_TOO_SMALL, "extract_mesh: %lld triangles, capacity %lld", (long long)n,
                    (long long)cap_tris);
    return MAP_OK;
}

extern "C" int map_set_schedule(map_t *m, int32_t tsdf, int32_t labels, int32_t mesh)
{
    if (!m) return MAP_ERR_INVALID_ARG;
    FLUSH_PENDING(m);
    const int v[3] = {tsdf, labels, mesh};
    for (int i = 0; i < 3; ++i)
        if (v[i] != 0 && v[i] != 1) return fail(m, MAP_ERR_INVALID_ARG, "set_schedule: schedules are 0 or 1");
    for (int i = 0; i < 3; ++i) m->sched[i] = v[i];
    set_bits(m);  // the counting grid may differ between meshing schedules
    return MAP_OK;
}

extern "C" int map_set_dirty_bitmap(map_t *m, int64_t min_blocks)
{
    if (!m) return MAP_ERR_INVALID_ARG;
    FLUSH_PENDING(m);  // a pending frame keeps the threshold it was enqueued under
    m->bits_user = min_blocks < 0 ? -1 : min_blocks;
    set_bits(m);
    return MAP_OK;
}

extern "C" int map_range_image(map_t *m, const lidar_model *L, const float *pts_dev, int64_t n, float F, float O,
                               float *depth_dev, float *height_dev, void *stream)
{
    if (!m) return MAP_ERR_INVALID_ARG;
    FLUSH_PENDING(m);
    if (!L || !L->elev_rad || !depth_dev || n < 0 || n > INT32_MAX || (n > 0 && !pts_dev))
        return fail(m, MAP_ERR_INVALID_ARG, "range_image: bad arguments");
    if (!std::isfinite(F) || !std::isfinite(O)) return fail(m, MAP_ERR_INVALID_ARG, "range_image: F and O must be finite");
    if (L->rows < 2 || L->cols < 8 || (int64_t)L->rows * L->cols > INT32_MAX)
        return fail(m, MAP_ERR_INVALID_ARG, "range_image: need rows >= 2, cols >= 8, rows * cols < 2^31");
    if (!(L->r_max > 0.0f) || !std::isfinite(L->r_max))
        return fail(m, MAP_ERR_INVALID_ARG, "range_image: r_max must be positive and finite");
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(m, hipSetDevice(m->p.device));
    const int rc = ensure_lut(m, L, s);
    if (rc) return rc;
    const int64_t npix = (int64_t)L->rows * L->cols;
    if (npix > m->rkeys_n) {
        HIP_TRY(m, hipDeviceSynchronize());  // an earlier call may still use the old keys
        if (m->rkeys) HIP_TRY(m, hipFree(m->rkeys));
        m->rkeys = nullptr;
        m->rkeys_n = 0;
        HIP_TRY(m, hipMalloc(&m->rkeys, (size_t)npix * sizeof(unsigned long long)));
        m->rkeys_n = npix;
        m->rkeys_dirty = true;
    }
    if (m->rkeys_dirty) HIP_TRY(m, launch_fill_u64(m->rkeys, (size_t)m->rkeys_n, ~0ull, s));
    m->rkeys_dirty = true;
    HIP_TRY(m, timed(m, MAP_K_RANGE, s, [&] {
        return launch_range_image(m->lut, pts_dev, (int)n, F, O, m->rkeys, depth_dev, height_dev, s);
    }));
    m->rkeys_dirty = false;
    m->last_stream = s;
    return MAP_OK;
}

extern "C" int map_query_sdf(map_t *m, const float *pts_dev, int64_t n, float *sdf_dev, float *grad_dev,
                             uint8_t *valid_dev, void *stream)
{
    if (!m) return MAP_ERR_INVALID_ARG;
    FLUSH_PENDING(m);
    if (n < 0 || (n > 0 && (!pts_dev || !sdf_dev || !valid_dev)))
        return fail(m, MAP_ERR_INVALID_ARG, "query_sdf: bad arguments");
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(m, hipSetDevice(m->p.device));
    HIP_TRY(m, timed(m, MAP_K_QUERY, s, [&] { return launch_query(m->v, pts_dev, n, sdf_dev, grad_dev, valid_dev, s); }));
    m->last_stream = s;
    return MAP_OK;
}

extern "C" int map_sdf_pose_adjoint(map_t *m, const float *xi_dev, const float *pts_dev, int32_t B, int64_t N,
                                    float *loss_dev, float *gxi_dev, float *gpts_dev, void *stream)
{
    if (!m) return MAP_ERR_INVALID_ARG;
    FLUSH_PENDING(m);
    if (B < 1 || B > 65535 || N < 1 || !xi_dev || !pts_dev || !loss_dev || !gxi_dev)
        return fail(m, MAP_ERR_INVALID_ARG, "sdf_pose_adjoint: bad arguments");
    const int64_t nchunk = (N + 255) / 256;
    if (nchunk > (int64_t)1 << 31) return fail(m, MAP_ERR_INVALID_ARG, "sdf_pose_adjoint: N too large");
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(m, hipSetDevice(m->p.device));
    const size_t need = (size_t)B * nchunk * 8;
    if (need > m->partial_floats) {
        HIP_TRY(m, hipStreamSynchronize(m->last_stream));
        HIP_TRY(m, hipStreamSynchronize(s));
        if (m->partial) HIP_TRY(m, hipFree(m->partial));
        m->partial = nullptr;
        HIP_TRY(m, hipMalloc(&m->partial, need * sizeof(float)));
        m->partial_floats = need;
    }
    HIP_TRY(m, timed(m, MAP_K_ADJOINT, s, [&] {
        hipError_t e = launch_adjoint(m->v, xi_dev, pts_dev, B, N, gpts_dev, m->partial, (int)nchunk, s);
        return e != hipSuccess ? e : launch_adjoint_reduce(xi_dev, m->partial, B, (int)nchunk, loss_dev, gxi_dev, s);
    }));
    m->last_stream = s;
    return MAP_OK;
}

// ---------------------------------------------------------------------------------
// map-quality metrics (Sec. V-C, Eq. 7, Eq. 8)
// ---------------------------------------------------------------------------------

namespace {
struct DevBuffers {  // device scratch of one call, freed on every return path
    std::vector<void *> ptrs;
    ~DevBuffers()
    {
        for (void *p : ptrs) (void)hipFree(p);
    }
    template <class T>
    hipError_t get(T **out, size_t count)
    {
        *out = nullptr;
        void *p = nullptr;
        const hipError_t e = hipMalloc(&p, std::max<size_t>(count, 1) * sizeof(T));
        if (e == hipSuccess) {
            ptrs.push_back(p);
            *out = static_cast<T *>(p);
        }
        return e;
    }
};
}  // namespace

extern "C" int map_mesh_quality(const float *mesh_pts_dev, const uint8_t *mesh_lab_dev, int64_t n_mesh,
                                const float *gt_pts_dev, const uint8_t *gt_lab_dev, int64_t n_gt, float voxel_size,
                                int32_t n_classes, int32_t device, double *d_mesh_dev, double *d_gt_dev,
                                int64_t *nn_gt_dev, int64_t *confusion_host, map_quality *out, void *stream)
{
    if (!out || n_mesh < 0 || n_gt < 0 || n_mesh > INT32_MAX || n_gt > INT32_MAX ||
        (n_mesh > 0 && (!mesh_pts_dev || !mesh_lab_dev)) || (n_gt > 0 && (!gt_pts_dev || !gt_lab_dev)))
        return fail(nullptr, MAP_ERR_INVALID_ARG, "mesh_quality: bad arguments");
    if (!(voxel_size > 0.0f) || !std::isfinite(voxel_size) || n_classes < 1 || n_classes > 254)
        return fail(nullptr, MAP_ERR_INVALID_ARG, "mesh_quality: need voxel_size > 0 and n_classes in [1, 254]");
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev)
        return fail(nullptr, MAP_ERR_INVALID_ARG, "mesh_quality: device %d not available", device);
#define Q_TRY(expr)                                                                                         \
    do {                                                                                                    \
        hipError_t e_ = (expr);                                                                             \
        if (e_ != hipSuccess)                                                                               \
            return fail(nullptr, MAP_ERR_DEVICE, "mesh_quality: %s: %s", #expr, hipGetErrorString(e_));      \
    } while (0)
    Q_TRY(hipSetDevice(device));
    hipStream_t s = (hipStream_t)stream;
    const double cap = 2.0 * (double)voxel_size;
    DevBuffers buf;
    // a grid per cloud: cells a little larger than the cap, so every point within the cap
    // of a query lies in one of the 27 cells around it whatever the rounding of x / h
    auto make_grid = [&](CellGrid &g, const float *p, int64_t n) -> hipError_t {
        const uint64_t slots = next_pow2(std::max<uint64_t>(2 * (uint64_t)n, 1024));
        g.mask = (uint32_t)(slots - 1);
        g.inv_h = 1.0 / (cap * (1.0 + 1e-6));
        hipError_t e;
        if ((e = buf.get(&g.key, slots)) != hipSuccess || (e = buf.get(&g.count, slots)) != hipSuccess ||
            (e = buf.get(&g.offset, slots)) != hipSuccess || (e = buf.get(&g.cursor, slots)) != hipSuccess ||
            (e = buf.get(&g.slot_of, (size_t)n)) != hipSuccess || (e = buf.get(&g.pts, (size_t)n)) != hipSuccess)
            return e;
        uint32_t *scan_tmp = nullptr;
        if ((e = buf.get(&scan_tmp, (slots + 255) / 256)) != hipSuccess) return e;
        if ((e = hipMemsetAsync(g.key, 0xFF, slots * sizeof(unsigned long long), s)) != hipSuccess) return e;
        if ((e = hipMemsetAsync(g.count, 0, slots * sizeof(uint32_t), s)) != hipSuccess) return e;
        if ((e = hipMemsetAsync(g.cursor, 0, slots * sizeof(uint32_t), s)) != hipSuccess) return e;
        return launch_grid_build(g, p, n, scan_tmp, s);
    };
    double *dM = d_mesh_dev, *dG = d_gt_dev;
    long long *nnG = reinterpret_cast<long long *>(nn_gt_dev);
    if (!dM) Q_TRY(buf.get(&dM, (size_t)n_mesh));
    if (!dG) Q_TRY(buf.get(&dG, (size_t)n_gt));
    if (!nnG) Q_TRY(buf.get(&nnG, (size_t)n_gt));
    CellGrid gG{}, gM{};
    Q_TRY(make_grid(gG, gt_pts_dev, n_gt));
    Q_TRY(launch_grid_query(gG, mesh_pts_dev, n_mesh, cap, dM, nullptr, s));
    Q_TRY(make_grid(gM, mesh_pts_dev, n_mesh));
    Q_TRY(launch_grid_query(gM, gt_pts_dev, n_gt, cap, dG, nnG, s));
    const int L = n_classes;
    const int nparts = (int)std::min<int64_t>(1024, std::max<int64_t>(1, (std::max(n_mesh, n_gt) + 255) / 256));
    double *partial = nullptr, *res = nullptr;
    unsigned long long *conf = nullptr;
    Q_TRY(buf.get(&partial, (size_t)nparts * 4));
    Q_TRY(buf.get(&res, 6));
    Q_TRY(buf.get(&conf, (size_t)(L + 1) * L));
    Q_TRY(hipMemsetAsync(conf, 0, (size_t)(L + 1) * L * sizeof(unsigned long long), s));
    Q_TRY(launch_quality(dM, n_mesh, dG, nnG, n_gt, mesh_lab_dev, gt_lab_dev, L, cap, partial, nparts, conf, res, s));
    double h_res[6];
    Q_TRY(hipMemcpyAsync(h_res, res, sizeof(h_res), hipMemcpyDeviceToHost, s));
    if (confusion_host)
        Q_TRY(hipMemcpyAsync(confusion_host, conf, (size_t)(L + 1) * L * sizeof(int64_t), hipMemcpyDeviceToHost, s));
    Q_TRY(hipStreamSynchronize(s));
#undef Q_TRY
    out->re = h_res[0];
    out->cd = h_res[1];
    out->rc = h_res[2];
    out->miou = h_res[3];
    out->acc = h_res[4];
    out->n_eval = (int64_t)h_res[5];
    return MAP_OK;
}

extern "C" int map_sdf_pose_adjoint_noalloc(map_t *m, const float *xi_dev, const float *pts_dev, int32_t B, int64_t N,
                                            float *loss_dev, float *gxi_dev, float *gpts_dev, void *stream)
{
    if (!m) return MAP_ERR_INVALID_ARG;
    FLUSH_PENDING(m);
    if (B < 1 || B > 65535 || N < 1 || !xi_dev || !pts_dev || !loss_dev || !gxi_dev)
        return fail(m, MAP_ERR_INVALID_ARG, "sdf_pose_adjoint_noalloc: bad arguments");
    const int64_t nchunk = (N + 255) / 256;
    if ((uint64_t)B * (uint64_t)nchunk * 8 > kScratchFloats)
        return fail(m, MAP_ERR_INVALID_ARG,
                    "sdf_pose_adjoint_noalloc: B * ceil(N / 256) = %lld exceeds the static scratch (%lld chunks)",
                    (long long)B * nchunk, (long long)(kScratchFloats / 8));
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(m, hipSetDevice(m->p.device));
    hipError_t se;
    float *part = scratch_on(m->p.device, &se);
    if (!part) return fail(m, MAP_ERR_DEVICE, "sdf_pose_adjoint_noalloc: scratch address: %s", hipGetErrorString(se));
    // launched directly: the kernel-event timer creates events, which this call must not
    HIP_TRY(m, launch_adjoint(m->v, xi_dev, pts_dev, B, N, gpts_dev, part, (int)nchunk, s));
    HIP_TRY(m, launch_adjoint_reduce(xi_dev, part, B, (int)nchunk, loss_dev, gxi_dev, s));
    m->last_stream = s;
    return MAP_OK;
}

static int read_counters(map_t *m)
{
    FLUSH_PENDING(m);
    HIP_TRY(m, hipSetDevice(m->p.device));
    HIP_TRY(m, hipStreamSynchronize(m->last_stream));
    HIP_TRY(m, hipMemcpy(m->h_ctr, m->v.ctr, sizeof(Counters), hipMemcpyDeviceToHost));
    return MAP_OK;
}

static int take_status(map_t *m)
{
    int st = m->h_ctr->status;
    if (st != 0) {
        int zero = 0;
        HIP_TRY(m, hipMemcpy((char *)m->v.ctr + offsetof(Counters, status), &zero, sizeof(int), hipMemcpyHostToDevice));
        return fail(m, st, "a LiDAR frame was rejected: it would exceed max_blocks");
    }
    return MAP_OK;
}

extern "C" int map_sync(map_t *m)
{
    if (!m) return MAP_ERR_INVALID_ARG;
    int rc = read_counters(m);
    if (rc) return rc;
    return take_status(m);
}

extern "C" int map_stats(map_t *m, map_frame_stats *out)
{
    if (!m || !out) return MAP_ERR_INVALID_ARG;
    int rc = read_counters(m);
    if (rc) return rc;
    const Counters &c = *m->h_ctr;
    out->touched = c.last_touched;
    out->new_blocks = c.last_new;
    out->updates = (int64_t)c.last_updates;
    Spread votes;
    HIP_TRY(m, hipMemcpy(&votes, &m->v.sync->votes, sizeof(Spread), hipMemcpyDeviceToHost));
    unsigned long long nv = 0;
    for (int l = 0; l < kLeaves; ++l) nv += votes.v[l * kLeafPad];
    out->votes = (int64_t)nv;
    out->mesh_blocks = (int64_t)c.mesh_blocks;
    out->triangles = (int64_t)c.mesh_tris;
    out->allocated = c.pool_used;
    out->frames = c.frames;
    out->mesh_from_bitmap = c.mesh_bits;
    return take_status(m);
}

extern "C" int64_t map_block_coords(map_t *m, int32_t *coords_host, int64_t cap)
{
    if (!m || read_counters(m)) return -1;
    const int64_t n = m->h_ctr->pool_used;
    const int64_t k = std::min(n, cap);
    if (k > 0 && coords_host) {
        std::vector<int4> tmp(k);
        if (hipMemcpy(tmp.data(), m->v.coords, k * sizeof(int4), hipMemcpyDeviceToHost) != hipSuccess) return -1;
        for (int64_t i = 0; i < k; ++i) {
            coords_host[3 * i] = tmp[i].x;
            coords_host[3 * i + 1] = tmp[i].y;
            coords_host[3 * i + 2] = tmp[i].z;
        }
    }
    return n;
}

extern "C" int64_t map_touched_coords(map_t *m, int32_t *coords_host, int64_t cap)
{
    if (!m || read_counters(m)) return -1;
    const int64_t n = m->h_ctr->last_touched;
    const int64_t k = std::min(n, cap);
    if (k > 0 && coords_host) {
        std::vector<unsigned long long> tmp(k);
        if (hipMemcpy(tmp.data(), m->f.tk_key, k * sizeof(unsigned long long), hipMemcpyDeviceToHost) != hipSuccess)
            return -1;
        for (int64_t i = 0; i < k; ++i) {
            int3 b = unpack_key(tmp[i]);
            coords_host[3 * i] = b.x;
            coords_host[3 * i + 1] = b.y;
            coords_host[3 * i + 2] = b.z;
        }
    }
    return n;
}

// Bulk download of the first min(cap, allocated) pool slots (tests and benchmarks).
extern "C" int64_t map_download(map_t *m, int64_t cap, int32_t *coords, float *D, float *W, uint8_t *fused,
                                uint16_t *counts)
{
    if (!m || read_counters(m)) return -1;
    const int64_t n = m->h_ctr->pool_used;
    const int64_t k = std::min(n, cap);
    if (k <= 0) return n;
    if (coords && map_block_coords(m, coords, k) < 0) return -1;
    if (D || W) {
        std::vector<float2> tmp((size_t)k * kBlockVoxels);
        if (hipMemcpy(tmp.data(), m->v.dw, tmp.size() * sizeof(float2), hipMemcpyDeviceToHost) != hipSuccess)
            return -1;
        for (size_t i = 0; i < tmp.size(); ++i) {
            if (D) D[i] = tmp[i].x;
            if (W) W[i] = tmp[i].y;
        }
    }
    if (fused && hipMemcpy(fused, m->v.fused, (size_t)k * kBlockVoxels, hipMemcpyDeviceToHost) != hipSuccess) return -1;
    if (counts && hipMemcpy(counts, m->v.counts, (size_t)k * m->p.n_classes * kBlockVoxels * sizeof(uint16_t),
                            hipMemcpyDeviceToHost) != hipSuccess)
        return -1;
    return n;
}

extern "C" int64_t map_download_aux(map_t *m, int64_t cap, float *grad, float *logpost)
{
    if (!m || read_counters(m)) return -1;
    const int64_t n = m->h_ctr->pool_used;
    const int64_t k = std::min(n, cap);
    if (k <= 0) return n;
    const size_t gb = (size_t)k * 3 * kBlockVoxels * sizeof(float);
    const size_t lb = (size_t)k * m->p.n_classes * kBlockVoxels * sizeof(float);
    if (grad) {
        if (m->v.grad) {
            if (hipMemcpy(grad, m->v.grad, gb, hipMemcpyDeviceToHost) != hipSuccess) return -1;
        } else {
            std::memset(grad, 0, gb);
        }
    }
    if (logpost) {
        if (m->v.logpost) {
            if (hipMemcpy(logpost, m->v.logpost, lb, hipMemcpyDeviceToHost) != hipSuccess) return -1;
        } else {
            std::memset(logpost, 0, lb);
        }
    }
    return n;
}

extern "C" int64_t map_frame_normals(map_t *m, float *out, int64_t cap)
{
    if (!m || read_counters(m)) return -1;
    if (m->dist_mode != kDistNonProjective || !m->f.nimg) return 0;
    const int64_t n = (int64_t)m->lut_rows * m->lut_cols;
    const int64_t k = std::min(n, cap);
    if (k > 0 && out && hipMemcpy(out, m->f.nimg, (size_t)k * sizeof(float4), hipMemcpyDeviceToHost) != hipSuccess)
        return -1;
    return n;
}

extern "C" int map_read_block(map_t *m, int32_t bx, int32_t by, int32_t bz, float *D, float *W, uint8_t *fused,
                              uint16_t *counts)
{
    if (!m || read_counters(m)) return 0;
    const int64_t n = m->h_ctr->pool_used;
    std::vector<int4> c(n > 0 ? n : 1);
    if (n > 0 && hipMemcpy(c.data(), m->v.coords, n * sizeof(int4), hipMemcpyDeviceToHost) != hipSuccess) return 0;
    for (int64_t i = 0; i < n; ++i) {
        if (c[i].x != bx || c[i].y != by || c[i].z != bz) continue;
        if (D || W) {
            float2 tmp[kBlockVoxels];
            if (hipMemcpy(tmp, m->v.dw + i * kBlockVoxels, sizeof(tmp), hipMemcpyDeviceToHost) != hipSuccess) return 0;
            for (int j = 0; j < kBlockVoxels; ++j) {
                if (D) D[j] = tmp[j].x;
                if (W) W[j] = tmp[j].y;
            }
        }
        if (fused && hipMemcpy(fused, m->v.fused + i * kBlockVoxels, kBlockVoxels, hipMemcpyDeviceToHost) != hipSuccess)
            return 0;
        const size_t cb = (size_t)m->p.n_classes * kBlockVoxels;
        if (counts && hipMemcpy(counts, m->v.counts + i * cb, cb * sizeof(uint16_t), hipMemcpyDeviceToHost) != hipSuccess)
            return 0;
        return 1;
    }
    return 0;
}

// ---------------------------------------------------------------------------------
// batched steps
// ---------------------------------------------------------------------------------

struct map_batch_s {
    std::vector<map_t *> maps;
    int device = 0;
    BatchMap *d_desc = nullptr, *h_desc = nullptr;
    BatchCtl *d_ctl = nullptr, *h_ctl = nullptr;
    BatchSync *d_sync = nullptr;
    MeshScan scan{};  // [kMaxMeshGrid][kMaxBatchMaps]
    MeshReport *h_reports = nullptr, *d_reports = nullptr;  // host-mapped, one per map of a step
    hipEvent_t done = nullptr;
    int schedule = 0, grid = 2048;
    bool use_graph = true;
    // one executable graph per step shape (map count, tile count, schedule, grid, stream)
    std::map<std::tuple<int, int, int, int, hipStream_t>, hipGraphExec_t> graphs;
    // the concurrent schedule: streams the maps' own kernel chains are spread over, and the
    // events that fork them from and join them to the caller's stream
    std::vector<hipStream_t> streams;
    std::vector<hipEvent_t> joins;
    hipEvent_t fork = nullptr;
    std::string err;
};

static void batch_free(map_batch_t *b)
{
    for (auto &g : b->graphs) (void)hipGraphExecDestroy(g.second);
    b->graphs.clear();
    for (hipStream_t st : b->streams) (void)hipStreamDestroy(st);
    for (hipEvent_t e : b->joins) (void)hipEventDestroy(e);
    if (b->fork) (void)hipEventDestroy(b->fork);
    b->streams.clear();
    b->joins.clear();
    if (b->d_desc) (void)hipFree(b->d_desc);
    if (b->d_ctl) (void)hipFree(b->d_ctl);
    void *ptrs[] = {b->d_sync, b->scan.wg_tris, b->scan.wg_blocks, b->scan.wg_off};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    if (b->h_reports) (void)hipHostFree(b->h_reports);
    if (b->done) (void)hipEventDestroy(b->done);
    if (b->h_desc) (void)hipHostFree(b->h_desc);
    if (b->h_ctl) (void)hipHostFree(b->h_ctl);
}

extern "C" int map_batch_create(map_t *const *maps, int32_t n, map_batch_t **out)
{
    if (!maps || !out || n < 1 || n > kMaxBatchMaps)
        return fail(nullptr, MAP_ERR_INVALID_ARG, "map_batch_create: need 1..%d maps", kMaxBatchMaps);
    *out = nullptr;
    for (int i = 0; i < n; ++i) {
        if (!maps[i]) return fail(nullptr, MAP_ERR_INVALID_ARG, "map_batch_create: NULL map %d", i);
        if (maps[i]->p.device != maps[0]->p.device)
            return fail(nullptr, MAP_ERR_INVALID_ARG, "map_batch_create: maps on different devices");
        for (int j = 0; j < i; ++j)
            if (maps[j] == maps[i]) return fail(nullptr, MAP_ERR_INVALID_ARG, "map_batch_create: map %d repeated", i);
    }
    map_batch_t *b = new map_batch_s();
    b->maps.assign(maps, maps + n);
    b->device = maps[0]->p.device;
    bool ok = hipSetDevice(b->device) == hipSuccess &&
              hipMalloc(&b->d_desc, kMaxBatchMaps * sizeof(BatchMap)) == hipSuccess &&
              hipMalloc(&b->d_ctl, sizeof(BatchCtl)) == hipSuccess &&
              hipMalloc(&b->d_sync, sizeof(BatchSync)) == hipSuccess &&
              hipMalloc(&b->scan.wg_tris, (size_t)kMaxMeshGrid * kMaxBatchMaps * sizeof(long long)) == hipSuccess &&
              hipMalloc(&b->scan.wg_blocks, (size_t)kMaxMeshGrid * kMaxBatchMaps * sizeof(int32_t)) == hipSuccess &&
              hipMalloc(&b->scan.wg_off, (size_t)kMaxMeshGrid * kMaxBatchMaps * sizeof(long long)) == hipSuccess &&
              hipHostMalloc((void **)&b->h_desc, kMaxBatchMaps * sizeof(BatchMap), hipHostMallocDefault) == hipSuccess &&
              hipHostMalloc((void **)&b->h_ctl, sizeof(BatchCtl), hipHostMallocDefault) == hipSuccess &&
              hipHostMalloc((void **)&b->h_reports, kMaxBatchMaps * sizeof(MeshReport),
                            hipHostMallocMapped | hipHostMallocCoherent) == hipSuccess &&
              hipHostGetDevicePointer((void **)&b->d_reports, b->h_reports, 0) == hipSuccess &&
              hipEventCreateWithFlags(&b->done, hipEventDisableTiming) == hipSuccess;
    if (ok) std::memset(b->h_reports, 0, kMaxBatchMaps * sizeof(MeshReport));
    if (ok) {
        std::memset(b->h_ctl, 0, sizeof(BatchCtl));
        ok = hipMemcpy(b->d_ctl, b->h_ctl, sizeof(BatchCtl), hipMemcpyHostToDevice) == hipSuccess &&
             hipMemset(b->d_sync, 0, sizeof(BatchSync)) == hipSuccess;
    }
    if (!ok) {
        batch_free(b);
        delete b;
        return fail(nullptr, MAP_ERR_DEVICE, "map_batch_create: device allocation failed");
    }
    *out = b;
    return MAP_OK;
}

extern "C" int map_batch_configure(map_batch_t *b, int32_t schedule, int32_t grid, int32_t use_graph)
{
    if (!b || schedule < 0 || schedule > kBatchConcurrent) return MAP_ERR_INVALID_ARG;
    if (schedule == kBatchConcurrent ? (grid < 1 || grid > kMaxBatchStreams) : (grid < 64 || grid > kMaxMeshGrid))
        return MAP_ERR_INVALID_ARG;
    if (schedule == kBatchConcurrent) {  // its streams and events, created once
        if (hipSetDevice(b->device) != hipSuccess) return MAP_ERR_DEVICE;
        if (!b->fork && hipEventCreateWithFlags(&b->fork, hipEventDisableTiming) != hipSuccess) return MAP_ERR_DEVICE;
        while ((int)b->streams.size() < grid) {
            hipStream_t st = nullptr;
            hipEvent_t ev = nullptr;
            if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) return MAP_ERR_DEVICE;
            b->streams.push_back(st);
            if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) return MAP_ERR_DEVICE;
            b->joins.push_back(ev);
        }
    }
    b->schedule = schedule;
    b->grid = grid;
    b->use_graph = use_graph != 0;
    return MAP_OK;
}

// The concurrent schedule of a step: each map's own kernels (allocation, TSDF with its
// camera labels fused, the two meshing passes), exactly as its plain calls launch them,
// the maps spread over the batch's streams so that their latency-bound chains overlap:
// largest first, each to the stream with the least work so far, a map's work taken as its
// scan's pixels over its voxel area (the blocks a frame touches grow with both).  The
// streams wait for the caller's stream first and it waits for them after.
static hipError_t launch_concurrent(map_batch_t *b, const map_batch_item *items, int n, hipStream_t s)
{
    const int K = std::min(b->grid, n);
    std::vector<double> work(n), load(K, 0.0);
    std::vector<int> order(n), stream_of(n);
    for (int i = 0; i < n; ++i) {
        const double nu = b->maps[items[i].map_index]->p.voxel_size;
        work[i] = (double)items[i].lidar->rows * items[i].lidar->cols / (nu * nu);
        order[i] = i;
    }
    std::stable_sort(order.begin(), order.end(), [&](int a, int c) { return work[a] > work[c]; });
    for (int i : order) {
        const int k = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        stream_of[i] = k;
        load[k] += work[i];
    }
    hipError_t e = hipEventRecord(b->fork, s);
    for (int k = 0; k < K && e == hipSuccess; ++k) e = hipStreamWaitEvent(b->streams[k], b->fork, 0);
    for (int j = 0; j < n && e == hipSuccess; ++j) {
        const int i = order[j];
        map_t *m = b->maps[items[i].map_index];
        const BatchMap &d = b->h_desc[i];
        const hipStream_t sk = b->streams[stream_of[i]];
        e = launch_alloc(m->v, m->f, m->lut, d.T, d.range, m->dist_mode, m->cos_inc, sk);
        if (e == hipSuccess)
            e = launch_tsdf(m->v, m->f, m->lut, d.T, m->f.rcopy, d.frame_id, m->sched[0],
                            grid_for(m->f.tk_cap, 1, m->tsdf_grid), m->dist_mode, d.cams, m->label_mode, sk);
        const MeshGrid grid = mesh_grid(m->sched[2]);
        m->scan.rec_cap = (int32_t)((m->p.max_blocks + grid.count - 1) / grid.count + 256);
        if (e == hipSuccess) e = launch_mesh_count(m->v, 0, m->scan, m->sched[2], grid, !m->bits_relaid, sk);
        m->bits_relaid = false;
        if (e == hipSuccess) e = launch_mesh_finish(m->v, 0, d.out, m->scan, b->d_reports + i, m->sched[2], grid, sk);
        m->last_stream = sk;
    }
    for (int k = 0; k < K && e == hipSuccess; ++k) {
        e = hipEventRecord(b->joins[k], b->streams[k]);
        if (e == hipSuccess) e = hipStreamWaitEvent(s, b->joins[k], 0);
    }
    return e;
}

extern "C" void map_batch_destroy(map_batch_t *b)
{
    if (!b) return;
    (void)hipSetDevice(b->device);
    (void)hipDeviceSynchronize();
    batch_free(b);
    delete b;
}

extern "C" int map_batch_step(map_batch_t *b, const map_batch_item *items, int32_t n, int64_t *n_tris, void *stream)
{
    if (!b || !items || !n_tris || n < 1 || n > (int)b->maps.size()) return MAP_ERR_INVALID_ARG;
    hipStream_t s = (hipStream_t)stream;
    if (hipSetDevice(b->device) != hipSuccess) return MAP_ERR_DEVICE;
    std::vector<char> seen(b->maps.size(), 0);
    // validate every item before touching any map (same checks as the plain calls)
    for (int i = 0; i < n; ++i) {
        const map_batch_item &it = items[i];
        if (it.map_index < 0 || it.map_index >= (int)b->maps.size() || seen[it.map_index]) {
            b->err = "map_batch_step: bad or repeated map index";
            return MAP_ERR_INVALID_ARG;
        }
        seen[it.map_index] = 1;
        map_t *m = b->maps[it.map_index];
        const lidar_model *L = it.lidar;
        if (!L || !L->elev_rad || !it.range_dev || !it.T_wl || L->rows < 2 || L->cols < 8 || !(L->r_max > 0.0f) ||
            !std::isfinite(L->r_max) || !pose_ok(it.T_wl) || it.n_cams < 0 || it.n_cams > kMaxCams ||
            (it.n_cams > 0 && (!it.cams || !it.labels_dev || !it.T_wc)) || it.cap_tris < 0 ||
            (it.cap_tris > 0 && (!it.pos_dev || !it.lab_dev))) {
            b->err = "map_batch_step: bad item";
            return fail(m, MAP_ERR_INVALID_ARG, "map_batch_step: bad item %d", i);
        }
        const double lim = (double)m->p.voxel_size * kDomainVoxels;
        for (int a = 0; a < 3; ++a)
            if (std::fabs((double)it.T_wl[4 * a + 3]) + (double)L->r_max + (double)m->p.truncation >= lim)
                return fail(m, MAP_ERR_INVALID_ARG, "map_batch_step: scan reaches outside the map domain");
        for (int c = 0; c < it.n_cams; ++c)
            if (!it.labels_dev[c] || !camera_ok(&it.cams[c]) || !pose_ok(it.T_wc + 16 * c))
                return fail(m, MAP_ERR_INVALID_ARG, "map_batch_step: bad camera %d of item %d", c, i);
        if (m->dist_mode != kDistProjective || m->label_mode != kLabelCounts)
            return fail(m, MAP_ERR_INVALID_ARG,
                        "map_batch_step: map %d is not in the plain modes (projective distance, vote counts)",
                        it.map_index);
    }
    for (map_t *m : b->maps) FLUSH_PENDING(m);
    int tiles = 0;
    for (int i = 0; i < n; ++i) {
        const map_batch_item &it = items[i];
        map_t *m = b->maps[it.map_index];
        int rc = ensure_lut(m, it.lidar, s);
        if (rc) return rc;
        rc = ensure_frame_scratch(m, it.lidar, s);
        if (rc) return rc;
        BatchMap &d = b->h_desc[i];
        d.v = m->v;
        d.f = m->f;
        d.lut = m->lut;
        d.T = to_pose(it.T_wl);
        d.range = it.range_dev;
        d.cams = CameraSet{};
        d.cams.n = it.n_cams;
        for (int c = 0; c < it.n_cams; ++c) {
            const camera_model &cm = it.cams[c];
            d.cams.cam[c] = Camera{cm.width, cm.height, cm.fx, cm.fy, cm.cx, cm.cy};
            d.cams.T[c] = to_pose(it.T_wc + 16 * c);
            d.cams.img[c] = it.labels_dev[c];
        }
        d.out = MeshOut{it.pos_dev, it.lab_dev, (long long *)it.edge_keys_dev, (long long)it.cap_tris};
        d.tile0 = tiles;
        d.tiles = (it.lidar->rows * it.lidar->cols + 255) / 256;
        d.frame_id = m->frame_id++;
        tiles += d.tiles;
    }
    auto fail_b = [&](hipError_t e, const char *what) {
        b->err = std::string(what) + ": " + hipGetErrorString(e);
        return MAP_ERR_DEVICE;
    };
    // Report slots follow item order, so clear their sequence numbers (no device write to
    // them is pending: the previous step returned after all of its reports).
    for (int i = 0; i < n; ++i) __atomic_store_n(&b->h_reports[i].seq, 0ull, __ATOMIC_RELEASE);
    hipError_t e = hipSuccess;
    if (b->schedule == kBatchConcurrent) {
        e = launch_concurrent(b, items, n, s);
        if (e != hipSuccess) return fail_b(e, "concurrent launch");
    } else if ((e = hipMemcpyAsync(b->d_desc, b->h_desc, n * sizeof(BatchMap), hipMemcpyHostToDevice, s)) !=
               hipSuccess) {
        return fail_b(e, "descriptor upload");
    } else if (b->use_graph && s != nullptr) {  // the legacy default stream cannot be captured
        const auto key = std::make_tuple(n, tiles, b->schedule, b->grid, s);
        auto itg = b->graphs.find(key);
        if (itg == b->graphs.end()) {
            hipGraph_t g = nullptr;
            hipGraphExec_t ge = nullptr;
            e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
            if (e != hipSuccess) return fail_b(e, "graph capture");
            hipError_t le =
                launch_batch(b->d_desc, b->d_ctl, b->d_sync, b->scan, b->d_reports, n, tiles, b->schedule, b->grid, s);
            e = hipStreamEndCapture(s, &g);
            if (le != hipSuccess) return fail_b(le, "batched launch");
            if (e != hipSuccess) return fail_b(e, "graph capture end");
            e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            if (e != hipSuccess) return fail_b(e, "graph instantiate");
            itg = b->graphs.emplace(key, ge).first;
        }
        e = hipGraphLaunch(itg->second, s);
        if (e != hipSuccess) return fail_b(e, "graph launch");
    } else {
        e = launch_batch(b->d_desc, b->d_ctl, b->d_sync, b->scan, b->d_reports, n, tiles, b->schedule, b->grid, s);
        if (e != hipSuccess) return fail_b(e, "batched launch");
    }
    e = hipEventRecord(b->done, s);
    if (e != hipSuccess) return fail_b(e, "step event");
    for (int i = 0; i < n; ++i) {
        map_t *m = b->maps[items[i].map_index];
        const uint32_t seq = ++m->n_extract;
        e = wait_report(&b->h_reports[i], seq, b->done);
        if (e != hipSuccess) {
            for (int j = i; j < n; ++j) {
                map_t *mj = b->maps[items[j].map_index];
                mj->n_extract = (uint32_t)__atomic_load_n(&b->h_reports[j].seq, __ATOMIC_ACQUIRE);
            }
            return fail_b(e, "step");
        }
    }
    int rc = MAP_OK;
    for (int i = 0; i < n; ++i) {
        map_t *m = b->maps[items[i].map_index];
        const int64_t t = (int64_t)__atomic_load_n(&b->h_reports[i].tris, __ATOMIC_ACQUIRE);
        n_tris[i] = t;
        m->has_scan = true;
        m->last_stream = s;
        if (t > items[i].cap_tris) {
            fail(m, MAP_ERR_BUFFER_TOO_SMALL, "map_batch_step: %lld triangles, capacity %lld", (long long)t,
                 (long long)items[i].cap_tris);
            rc = MAP_ERR_BUFFER_TOO_SMALL;
        }
    }
    return rc;
}
