// C-ABI of the vbx TSDF integrator: map lifecycle, per-call scratch, the launch sequence of
// one integration call, and the cold paths (export, import, statistics).
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <deque>
#include <thread>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "../../include/vbx.h"
#include "vbx_host.h"
#include "vbx_internal.h"
#include "vbx_sched.h"

using namespace vbx;

// Scratch region of vbx_integrate_frames_noalloc: one copy per device, held for the life of the
// process.  In host code this name only stands for the symbol: its device address comes from
// hipGetSymbolAddress (NoAllocDevice below), and only that address is ever handed to a kernel.
static __device__ __align__(256) unsigned char scratch[VBX_NOALLOC_SCRATCH_BYTES];

namespace {

#define VBX_TRY(expr)                                  \
    do {                                               \
        hipError_t e_ = (expr);                        \
        if (e_ != hipSuccess) return VBX_ERR_DEVICE;   \
    } while (0)

size_t next_pow2(size_t x) {
    size_t p = 1;
    while (p < x) p <<= 1;
    return p;
}

// A grow-only device buffer.
struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
};

// Pinned staging for the per-call job and map tables, in a small ring so that a call never
// overwrites a table whose copy to the device is still queued.
struct Stage {
    void* host = nullptr;
    size_t bytes = 0;
    hipEvent_t ev = nullptr;
    bool used = false;
};

struct Scratch {
    DevBuf rays_p, rays_job, cross, ncross, sorted, tkeys, tval, tlist, t_key, t_slot, order, bins, off,
        partial, parts, parts_sorted, tile_parts, chunk_first, touch_key, touch_n, tables, jst, cs;
    DevBuf hbins;   // crossing counts by (block-set slot, frame), kept zero between calls
    DevBuf rays_c, sorted_c, parts_c, parts_sorted_c;   // colour calls: the colours beside the rays
    size_t ray_cap = 0, cross_cap = 0, tkey_cap = 0, tlist_cap = 0, bins_cap = 0, nparts = 0,
           touch_cap = 0, hbins_cap = 0;
    Stage stage[4];
    int stage_i = 0;
    // host copy of the maps of the last call (for vbx_last_touches)
    std::vector<vbx_map*> last_maps;
    bool touches_valid = false;
};

}  // namespace

// Per-stage event timing of a map's calls.
struct Profiler {
    struct Rec {
        int stage;
        hipEvent_t a, b;
    };
    u32 mask = 0;   // stages whose launches are timed (bit i: stage i)
    std::vector<hipEvent_t> spare;
    std::vector<Rec> pending;
    double ms[VBX_PROFILE_STAGES] = {};
    uint64_t launches[VBX_PROFILE_STAGES] = {};
    hipEvent_t take() {
        if (!spare.empty()) {
            hipEvent_t e = spare.back();
            spare.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        return e;
    }
};

enum { ST_POINTS, ST_GROUPS, ST_CROSS, ST_RESOLVE, ST_COMMIT, ST_BINS, ST_SCAN, ST_SCATTER, ST_UPDATE, ST_FINISH };

// A map's ESDF layer (host side).  The voxel words cover the pool slots [0, vox_blocks), grown
// with the map; the dirty flags cover the whole pool.
struct Esdf {
    vbx_esdf_params P;
    u64* vox = nullptr;          // map memory: [vox_blocks * 4096]
    size_t vox_blocks = 0;
    u32* dirty = nullptr;        // map memory: [dirty_cap]
    u32 dirty_cap = 0;
    DevBuf rstamp, lstamp, list, nbr, slot_key, raise0, raise1, lower0, lower1, cnt;
    u32 tag = 0;                 // last frontier tag handed out (tags only grow)
    u32 nbr_blocks = 0;          // blocks the neighbour tables were built for (0: rebuild)
    vbx_esdf_stats stats = {};
};

struct vbx_map {
    vbx_map_params P;
    Profiler prof;
    int device = 0;
    hipStream_t stream = nullptr;
    MapState* st = nullptr;       // device
    u64* hkeys = nullptr;         // device
    int* hslots = nullptr;        // device
    u32 hcap = 0;
    void* pool = nullptr;         // device
    u32* color = nullptr;         // device, VBX_FLAG_COLOR: [capacity][4096] packed RGB8
    u32 capacity = 0;
    size_t voxel_bytes = 8;
    int wbits = 0;
    int kw = 0;
    Scratch* scratch = nullptr;
    Scratch* touch_src = nullptr; // scratch holding this map's last touches
    int touch_idx = 0;
    int update_variant = 6;       // index into kUpdateVariants (whole block, 1024 threads)
    Esdf* esdf = nullptr;         // ESDF layer, when enabled
};

// A captured call: the kernel sequence of one integration call over fixed maps and frame
// shapes, replayed with hipGraphLaunch.  It owns its scratch, so eager calls on the same maps
// never move buffers the graph refers to.
struct vbx_graph {
    std::vector<vbx_map*> maps;
    std::vector<int> owner;
    std::vector<vbx_frame> frames;   // frames of the next launch
    std::vector<u32> capacity;       // map capacities at capture
    size_t sum_capacity = 0;
    int update_variant = 1;
    Scratch* scratch = nullptr;
    hipStream_t capture_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace {

int dev_alloc(DevBuf& b, size_t bytes) {
    if (b.bytes >= bytes && b.p) return VBX_OK;
    if (b.p) {
        (void)hipFree(b.p);
        b.p = nullptr;
        b.bytes = 0;
    }
    if (bytes == 0) bytes = 256;
    if (hipMalloc(&b.p, bytes) != hipSuccess) {
        b.p = nullptr;
        return VBX_ERR_OUT_OF_MEMORY;
    }
    b.bytes = bytes;
    return VBX_OK;
}

unsigned grid_for(size_t n, unsigned cap = 2048) {
    size_t g = (n + 255) / 256;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (unsigned)g;
}

int weight_bits(const vbx_map_params& P) {
    if (P.weighting == VBX_W_CONST) return 0;
    const float wmax = 1.0f / (P.z_min * P.z_min);
    int c = 0;
    while (std::ldexp(1.0f, c) < wmax) ++c;
    return 32 - c;
}

// Fixed-point bits of the per-voxel weight sums: every (voxel, frame) sum stays below 2^62
// for frames of up to 2^24 points with weights up to 2^(32 - wbits).
int sum_bits(const vbx_map_params& P) {
    const int c = P.weighting == VBX_W_CONST ? 0 : 32 - weight_bits(P);
    return 38 - c;
}

// Length of a ray's walk in voxels: the truncation band, or the whole ray up to trunc behind a
// point at the maximum range.
double walk_voxels(const vbx_map_params& P) {
    const double len = (P.flags & VBX_FLAG_FULL_RAY) ? (double)P.max_range + (double)P.trunc : 2.0 * (double)P.trunc;
    return len / (double)P.voxel_size;
}

int max_blocks_per_ray(const vbx_map_params& P) {
    const double len = walk_voxels(P) + 2.0;
    return 1 + 3 * ((int)std::floor(len / 16.0) + 1);
}

int max_voxels_per_ray(const vbx_map_params& P) {
    return 3 * ((int)std::ceil(walk_voxels(P)) + 2) + 1;
}

int validate_params(const vbx_map_params& P) {
    if (!(P.voxel_size > 0.0f) || !std::isfinite(P.voxel_size)) return VBX_ERR_INVALID_ARG;
    if (!(P.trunc > 0.0f) || !std::isfinite(P.trunc)) return VBX_ERR_INVALID_ARG;
    if (!(P.w_max > 0.0f)) return VBX_ERR_INVALID_ARG;
    if (!(P.max_range > 0.0f) || !std::isfinite(P.max_range)) return VBX_ERR_INVALID_ARG;
    if (P.weighting != VBX_W_CONST && P.weighting != VBX_W_QUAD) return VBX_ERR_INVALID_ARG;
    if (P.merge != VBX_MERGE_NONE && P.merge != VBX_MERGE_GROUPED) return VBX_ERR_INVALID_ARG;
    if (P.storage != VBX_F32 && P.storage != VBX_F16 && P.storage != VBX_S16) return VBX_ERR_INVALID_ARG;
    if (P.dist != VBX_DIST_EQ1 && P.dist != VBX_DIST_ALONG_RAY) return VBX_ERR_INVALID_ARG;
    if (P.weighting == VBX_W_QUAD && !(P.z_min >= 0.05f)) return VBX_ERR_INVALID_ARG;
    if (P.storage != VBX_F32 && P.w_max > 65504.0f) return VBX_ERR_INVALID_ARG;   // binary16 W
    if ((P.alloc == nullptr) != (P.free == nullptr)) return VBX_ERR_INVALID_ARG;
    if (P.block_capacity == 0 || P.block_capacity > (1u << 29)) return VBX_ERR_INVALID_ARG;
    if (2.0 * P.trunc / P.voxel_size > 28.0) return VBX_ERR_LIMIT;   // band of <= 28 voxels
    if ((P.flags & VBX_FLAG_FULL_RAY) && walk_voxels(P) > 1024.0) return VBX_ERR_LIMIT;
    return VBX_OK;
}

MapDesc make_desc(const vbx_map* m, int map_id, int job0, int njobs) {
    const vbx_map_params& P = m->P;
    MapDesc d;
    std::memset(&d, 0, sizeof d);
    d.v = P.voxel_size;
    d.iv = 1.0f / P.voxel_size;
    d.delta = P.trunc;
    d.inv_delta = 1.0f / P.trunc;
    {
        const float e = d.delta * d.inv_delta;   // binary32, as the kernels form d / delta
        d.e_max = e < 1.0f ? e : 1.0f;
    }
    d.eps = P.voxel_size;
    d.ramp = 1.0f / (P.trunc - P.voxel_size);
    d.w_max = P.w_max;
    d.rmax2 = P.max_range * P.max_range;
    d.z_min = P.z_min;
    d.wscale = std::ldexp(1.0f, m->kw);
    d.inv_wscale = std::ldexp(1.0f, -m->kw);
    d.weighting = P.weighting;
    d.merge = P.merge;
    d.storage = P.storage;
    d.dist = P.dist;
    d.wbits = m->wbits;
    d.njobs = njobs;
    d.job0 = job0;
    d.map_id = map_id;
    d.hkeys = m->hkeys;
    d.hslots = m->hslots;
    d.hmask = m->hcap - 1;
    d.capacity = m->capacity;
    d.pool = m->pool;
    d.st = m->st;
    d.dirty = m->esdf ? m->esdf->dirty : nullptr;
    d.full_ray = (P.flags & VBX_FLAG_FULL_RAY) ? 1 : 0;
    d.max_steps = max_voxels_per_ray(P) + 1;
    d.color = m->color;
    return d;
}

// The map's own device memory (hash table, block pool, device state): the caller's allocator
// hook when the parameters carry one, else hipMalloc / hipFree.
int map_alloc(const vbx_map* m, void** p, size_t bytes) {
    *p = nullptr;
    if (m->P.alloc) {
        *p = m->P.alloc(bytes, m->P.alloc_ctx);
        return *p ? VBX_OK : VBX_ERR_OUT_OF_MEMORY;
    }
    if (hipMalloc(p, bytes) != hipSuccess) {
        *p = nullptr;
        return VBX_ERR_OUT_OF_MEMORY;
    }
    return VBX_OK;
}

void map_free(const vbx_map* m, void* p) {
    if (!p) return;
    if (m->P.free) m->P.free(p, m->P.alloc_ctx);
    else (void)hipFree(p);
}

int alloc_storage(vbx_map* m, u32 capacity) {
    m->capacity = capacity;
    m->hcap = (u32)next_pow2((size_t)capacity * 2);
    if (map_alloc(m, (void**)&m->hkeys, sizeof(u64) * m->hcap) != VBX_OK) return VBX_ERR_OUT_OF_MEMORY;
    if (map_alloc(m, (void**)&m->hslots, sizeof(int) * m->hcap) != VBX_OK) return VBX_ERR_OUT_OF_MEMORY;
    if (map_alloc(m, &m->pool, (size_t)capacity * 4096 * m->voxel_bytes) != VBX_OK)
        return VBX_ERR_OUT_OF_MEMORY;
    if (m->P.flags & VBX_FLAG_COLOR) {
        if (map_alloc(m, (void**)&m->color, (size_t)capacity * 4096 * sizeof(u32)) != VBX_OK)
            return VBX_ERR_OUT_OF_MEMORY;
        // a slot's colour starts black: only the update of a colour call writes it afterwards
        hipLaunchKernelGGL(k_fill_u32, dim3(grid_for((size_t)capacity * 4096, 8192)), dim3(256), 0, m->stream,
                           m->color, 0u, (size_t)capacity * 4096);
    }
    hipLaunchKernelGGL(k_fill_u64, dim3(grid_for(m->hcap)), dim3(256), 0, m->stream, m->hkeys, kEmpty,
                       (size_t)m->hcap);
    return hipGetLastError() == hipSuccess ? VBX_OK : VBX_ERR_DEVICE;
}

void free_storage(vbx_map* m) {
    map_free(m, m->hkeys);
    map_free(m, m->hslots);
    map_free(m, m->pool);
    map_free(m, m->color);
    m->hkeys = nullptr;
    m->hslots = nullptr;
    m->pool = nullptr;
    m->color = nullptr;
}

// Colour maps: every slot back to black (after the map's blocks were replaced or dropped).
void clear_colors(vbx_map* m) {
    if (!m->color) return;
    const size_t n = (size_t)m->capacity * 4096;
    hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(n, 8192)), dim3(256), 0, m->stream, m->color, 0u, n);
}

void free_scratch(Scratch* s) {
    if (!s) return;
    DevBuf* bufs[] = {&s->rays_p, &s->rays_job, &s->cross, &s->ncross, &s->sorted, &s->tkeys,
                      &s->tval, &s->tlist, &s->t_key, &s->t_slot, &s->order, &s->bins, &s->off, &s->partial,
                      &s->parts, &s->parts_sorted, &s->tile_parts, &s->chunk_first, &s->touch_key, &s->touch_n,
                      &s->tables, &s->jst, &s->cs, &s->rays_c, &s->sorted_c, &s->parts_c,
                      &s->parts_sorted_c};
    for (DevBuf* b : bufs)
        if (b->p) (void)hipFree(b->p);
    for (Stage& st : s->stage) {
        if (st.host) (void)hipHostFree(st.host);
        if (st.ev) (void)hipEventDestroy(st.ev);
    }
    delete s;
}

struct CallPlan {
    size_t total_points = 0;
    size_t ray_slots = 0;       // tiles x points per tile
    u32 tiles = 0;
    int JM = 1;
    int max_blocks = 4;
    int max_vox = 22;
    bool grouped = false;
    int storage = 0;
    bool keep_touches = false;
    u32 tiles_per_job = 0;      // every job has this many tiles and there is one map (else 0)
    bool projective = false;    // projection mapping instead of raycasting the voxels
    Intrinsics K = {};          // its camera intrinsics
    bool color = false;         // a map of the call keeps colour: the rays carry colours
};

// Element counts of a call's scratch buffers (host upper bounds: nothing is read back mid-call).
struct ScratchSizes {
    size_t ray_cap, cross_cap, tlist_cap, tkey_cap, bins_cap, hbins_cap, nparts, touch_cap, tables_bytes;
};

int scratch_sizes(const CallPlan& plan, int njobs, int nmaps, size_t sum_capacity, ScratchSizes& z) {
    z.ray_cap = std::max<size_t>(plan.ray_slots, 1);
    z.cross_cap = z.ray_cap * (size_t)plan.max_blocks;
    if (z.cross_cap > 0xFFFFFFF0ull || z.ray_cap > 0xFFFFFFF0ull) return VBX_ERR_LIMIT;
    z.tlist_cap = std::min<size_t>(std::max<size_t>(sum_capacity + 4096, 4096), z.cross_cap + 4096);
    z.tkey_cap = next_pow2(2 * z.tlist_cap);
    // grouped calls sort partial groups into kGroupSubBins bins per (block, frame)
    z.bins_cap = z.tlist_cap * (size_t)plan.JM * (plan.grouped ? (size_t)kGroupSubBins : 1u);
    if (z.bins_cap > 0xFFFFFFF0ull) return VBX_ERR_LIMIT;
    // the crossing kernel counts crossings by (block-set slot, frame) before blocks have dense
    // indices; the scan moves the counts to dense order
    z.hbins_cap = z.tkey_cap * (size_t)plan.JM;
    if (z.hbins_cap > 0xFFFFFFF0ull) return VBX_ERR_LIMIT;
    z.nparts = (z.bins_cap + kScanChunkHost - 1) / kScanChunkHost;
    z.touch_cap = plan.keep_touches ? std::min<size_t>(z.ray_cap * (size_t)plan.max_vox, (size_t)1 << 26) : 0;
    if (plan.keep_touches && plan.projective)   // every voxel of every block of the call
        z.touch_cap = std::min<size_t>(z.tlist_cap * 4096, (size_t)1 << 26);
    z.tables_bytes = (size_t)nmaps * sizeof(MapDesc) + (size_t)njobs * sizeof(Job);
    return VBX_OK;
}

// Calls `f(buffer, bytes)` for every scratch buffer a call with sizes `z` uses, in one fixed order.
template <class F>
void for_each_scratch(Scratch* s, const CallPlan& plan, const ScratchSizes& z, int njobs, F&& f) {
    f(s->rays_p, z.ray_cap * sizeof(float4));
    f(s->rays_job, z.ray_cap * sizeof(u32));
    f(s->cross, z.cross_cap * sizeof(u32));
    f(s->ncross, z.ray_cap);
    f(s->sorted, z.cross_cap * sizeof(float4));
    f(s->tkeys, z.tkey_cap * sizeof(u64));
    f(s->tval, z.tkey_cap * sizeof(u32));
    f(s->tlist, z.tlist_cap * sizeof(u32));
    f(s->t_key, z.tlist_cap * sizeof(u64));
    f(s->t_slot, z.tlist_cap * sizeof(int));
    f(s->order, z.tlist_cap * sizeof(u32));
    f(s->bins, (z.bins_cap + 1) * sizeof(u32));
    f(s->hbins, z.hbins_cap * sizeof(u32));
    f(s->off, (z.bins_cap + 1) * sizeof(u32));
    f(s->partial, (z.nparts + 1) * sizeof(u32));
    if (plan.grouped) {
        // partial groups: a tile of kTileGrouped points owns kTileGrouped slots
        f(s->parts, z.ray_cap * sizeof(Partial));
        f(s->parts_sorted, z.ray_cap * sizeof(Partial));
        f(s->tile_parts, std::max<size_t>(plan.tiles, 1) * sizeof(u32));
        f(s->chunk_first, (z.ray_cap / kMergeSpan + 2) * sizeof(u32));
    }
    if (plan.color) {
        f(s->rays_c, z.ray_cap * sizeof(u32));
        f(s->sorted_c, z.cross_cap * sizeof(u32));
        if (plan.grouped) {
            f(s->parts_c, z.ray_cap * sizeof(PartialColor));
            f(s->parts_sorted_c, z.ray_cap * sizeof(PartialColor));
        }
    }
    if (plan.keep_touches) {
        f(s->touch_key, z.touch_cap * sizeof(u64));
        f(s->touch_n, z.touch_cap * sizeof(u32));
    }
    f(s->tables, z.tables_bytes);
    f(s->jst, (size_t)njobs * sizeof(JobStat));
    f(s->cs, sizeof(CallState));
}

void note_scratch_sizes(Scratch* s, const ScratchSizes& z) {
    s->ray_cap = z.ray_cap;
    s->cross_cap = z.cross_cap;
    s->tlist_cap = z.tlist_cap;
    s->bins_cap = z.bins_cap;
    s->hbins_cap = z.hbins_cap;
    s->nparts = z.nparts;
    s->tkey_cap = z.tkey_cap;
    s->touch_cap = z.touch_cap;
}

// Grows a scratch set for a call on stream `st`; tables that must start cleared are cleared here.
int ensure_scratch(Scratch* s, hipStream_t st, const CallPlan& plan, int njobs, int nmaps, size_t sum_capacity) {
    ScratchSizes z;
    int rc = scratch_sizes(plan, njobs, nmaps, sum_capacity, z);
    if (rc != VBX_OK) return rc;
    const size_t ray_cap = z.ray_cap, cross_cap = z.cross_cap, tlist_cap = z.tlist_cap, tkey_cap = z.tkey_cap,
                 bins_cap = z.bins_cap, nparts = z.nparts, touch_cap = z.touch_cap;

    bool need_sync = false;
    auto grow = [&](DevBuf& b, size_t bytes) -> int {
        if (b.bytes >= bytes && b.p) return 0;
        if (!need_sync) {
            (void)hipStreamSynchronize(st);
            need_sync = true;
        }
        return dev_alloc(b, bytes) == VBX_OK ? 1 : -1;
    };
    int r;
#define GROW(buf, bytes)                          \
    if ((r = grow(buf, bytes)) < 0) return VBX_ERR_OUT_OF_MEMORY;

    GROW(s->rays_p, ray_cap * sizeof(float4));
    GROW(s->rays_job, ray_cap * sizeof(u32));
    GROW(s->cross, cross_cap * sizeof(u32));
    GROW(s->ncross, ray_cap);
    GROW(s->sorted, cross_cap * sizeof(float4));
    if ((r = grow(s->tkeys, tkey_cap * sizeof(u64))) < 0) return VBX_ERR_OUT_OF_MEMORY;
    if (r == 1 || s->tkey_cap != tkey_cap) {
        hipLaunchKernelGGL(k_fill_u64, dim3(grid_for(tkey_cap)), dim3(256), 0, st, (u64*)s->tkeys.p,
                           kEmpty, tkey_cap);
    }
    s->tkey_cap = tkey_cap;
    GROW(s->tval, tkey_cap * sizeof(u32));
    GROW(s->tlist, tlist_cap * sizeof(u32));
    GROW(s->t_key, tlist_cap * sizeof(u64));
    GROW(s->t_slot, tlist_cap * sizeof(int));
    GROW(s->order, tlist_cap * sizeof(u32));
    if ((r = grow(s->bins, (bins_cap + 1) * sizeof(u32))) < 0) return VBX_ERR_OUT_OF_MEMORY;
    if (r == 1)
        hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(bins_cap + 1)), dim3(256), 0, st, (u32*)s->bins.p, 0u,
                           bins_cap + 1);
    if ((r = grow(s->hbins, z.hbins_cap * sizeof(u32))) < 0) return VBX_ERR_OUT_OF_MEMORY;
    if (r == 1)
        hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(s->hbins.bytes / 4)), dim3(256), 0, st, (u32*)s->hbins.p, 0u,
                           s->hbins.bytes / 4);
    s->hbins_cap = z.hbins_cap;
    GROW(s->off, (bins_cap + 1) * sizeof(u32));
    GROW(s->partial, (nparts + 1) * sizeof(u32));
    if (plan.grouped) {
        // partial groups: a tile of kTileGrouped points owns kTileGrouped slots
        GROW(s->parts, ray_cap * sizeof(Partial));
        GROW(s->parts_sorted, ray_cap * sizeof(Partial));
        GROW(s->tile_parts, std::max<size_t>(plan.tiles, 1) * sizeof(u32));
        GROW(s->chunk_first, (ray_cap / kMergeSpan + 2) * sizeof(u32));
    }
    if (plan.color) {
        GROW(s->rays_c, ray_cap * sizeof(u32));
        GROW(s->sorted_c, cross_cap * sizeof(u32));
        if (plan.grouped) {
            GROW(s->parts_c, ray_cap * sizeof(PartialColor));
            GROW(s->parts_sorted_c, ray_cap * sizeof(PartialColor));
        }
    }
    if (plan.keep_touches) {
        GROW(s->touch_key, touch_cap * sizeof(u64));
        GROW(s->touch_n, touch_cap * sizeof(u32));
        s->touch_cap = touch_cap;
    }
    const size_t tables_bytes = (size_t)nmaps * sizeof(MapDesc) + (size_t)njobs * sizeof(Job);
    GROW(s->tables, tables_bytes);
    if ((r = grow(s->jst, (size_t)njobs * sizeof(JobStat))) < 0) return VBX_ERR_OUT_OF_MEMORY;
    if (r == 1)
        hipLaunchKernelGGL(k_fill_u64, dim3(grid_for(s->jst.bytes / 8)), dim3(256), 0, st, (u64*)s->jst.p, 0ull,
                           s->jst.bytes / 8);
    if ((r = grow(s->cs, sizeof(CallState))) < 0) return VBX_ERR_OUT_OF_MEMORY;
    if (r == 1) hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(256), 0, st, (u32*)s->cs.p, 0u, sizeof(CallState) / 4);
#undef GROW
    s->ray_cap = ray_cap;
    s->cross_cap = cross_cap;
    s->tlist_cap = tlist_cap;
    s->bins_cap = bins_cap;
    s->nparts = nparts;
    return VBX_OK;
}

// Persistent grid of the group-merge kernel.
int group_merge_grid() {
    static int grid = 0;
    static std::once_flag once;
    std::call_once(once, [] {
        int dev = 0, cus = 256, per = 1;
        (void)hipGetDevice(&dev);
        (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, reinterpret_cast<const void*>(&k_group_merge<false>), 256, 0) !=
                hipSuccess || per < 1)
            per = 1;
        grid = cus * per;
    });
    return grid > 0 ? grid : 256;
}

// Workgroups of the crossing kernel that the chip holds at once (its LDS block set allows
// fewer per CU than the thread limit): a persistent grid of that many, since a larger grid
// runs its last workgroups in a second, mostly idle round.
unsigned cross_grid() {
    static unsigned grid = 0;
    static std::once_flag once;
    std::call_once(once, [] {
        int dev = 0, cus = 256, per = 1;
        (void)hipGetDevice(&dev);
        (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, reinterpret_cast<const void*>(&k_cross), 256, 0) !=
                hipSuccess || per < 1)
            per = 1;
        grid = (unsigned)cus * (unsigned)per;
    });
    return grid > 0 ? grid : 256u;
}

// Waves of the partial-group sort kernels that the chip holds at once.
unsigned sort_resident_waves() {
    static unsigned waves = 0;
    static std::once_flag once;
    std::call_once(once, [] {
        int dev = 0, cus = 256, per = 1;
        (void)hipGetDevice(&dev);
        (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, reinterpret_cast<const void*>(&k_gscatter), 256, 0) !=
                hipSuccess || per < 1)
            per = 1;
        waves = (unsigned)cus * (unsigned)per * 4u;
    });
    return waves > 0 ? waves : 8192u;
}

// Persistent grid of an update-kernel variant: one workgroup per slot the chip can hold.
template <int STORAGE, int RX, int RY, int RZ, int NT, bool COLOR = false>
int update_grid() {
    static int grid = 0;
    static std::once_flag once;
    std::call_once(once, [] {
        int dev = 0, cus = 256, per = 1;
        (void)hipGetDevice(&dev);
        (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
                &per, reinterpret_cast<const void*>(&k_update<STORAGE, RX, RY, RZ, NT, COLOR>), NT, 0) != hipSuccess ||
            per < 1)
            per = 1;
        grid = cus * per;
    });
    return grid > 0 ? grid : 256;
}

template <int STORAGE, int RX, int RY, int RZ, int NT, bool COLOR = false>
void launch_update_t(hipStream_t st, const Job* jobs, const MapDesc* maps, const u64* t_key,
                     const int* t_slot, const u32* off, const u32* order, const float4* sorted,
                     const u32* sorted_c, u32 JM, u64* touch_key, u32* touch_n, u32 touch_cap, int keep,
                     JobStat* jst, CallState* cs) {
    hipLaunchKernelGGL((k_update<STORAGE, RX, RY, RZ, NT, COLOR>),
                       dim3(update_grid<STORAGE, RX, RY, RZ, NT, COLOR>()), dim3(NT), 0, st, jobs, maps, t_key,
                       t_slot, off, order, sorted, sorted_c, JM, touch_key, touch_n, touch_cap, keep, jst, cs);
}

// Update-kernel variants: how a block is cut into regions, and the workgroup size.  Larger
// workgroups put more waves on the rays of one block (its frames fold in sequence, so a
// heavily observed block is a long chain for one workgroup).
struct UpdateVariant {
    int split;     // regions per block
    int columns;   // 0: z-slabs; 1: columns cut across x and y
    int threads;   // workgroup size
};
constexpr UpdateVariant kUpdateVariants[] = {{1, 0, 256}, {2, 0, 256}, {4, 0, 256}, {2, 1, 256}, {4, 1, 256},
                                             {8, 1, 256}, {1, 0, 1024}, {2, 0, 1024}, {4, 0, 1024}, {2, 0, 512}};
constexpr int kNumUpdateVariants = sizeof(kUpdateVariants) / sizeof(kUpdateVariants[0]);
static_assert(kNumUpdateVariants == VBX_TUNING_CANDIDATES, "tuning candidates");

template <int STORAGE>
void launch_update_s(int variant, hipStream_t st, const Job* jobs, const MapDesc* maps, const u64* t_key,
                     const int* t_slot, const u32* off, const u32* order, const float4* sorted, u32 JM,
                     u64* touch_key, u32* touch_n, u32 touch_cap, int keep, JobStat* jst, CallState* cs) {
#define VBX_UPD(X, Y, Z, T)                                                                        \
    launch_update_t<STORAGE, X, Y, Z, T>(st, jobs, maps, t_key, t_slot, off, order, sorted, nullptr, JM, touch_key, \
                                         touch_n, touch_cap, keep, jst, cs)
    switch (variant) {
        case 0: VBX_UPD(16, 16, 16, 256); break;
        case 2: VBX_UPD(16, 16, 4, 256); break;
        case 3: VBX_UPD(8, 16, 16, 256); break;
        case 4: VBX_UPD(8, 8, 16, 256); break;
        case 5: VBX_UPD(4, 8, 16, 256); break;
        case 6: VBX_UPD(16, 16, 16, 1024); break;
        case 7: VBX_UPD(16, 16, 8, 1024); break;
        case 8: VBX_UPD(16, 16, 4, 1024); break;
        case 9: VBX_UPD(16, 16, 8, 512); break;
        default: VBX_UPD(16, 16, 8, 256); break;
    }
#undef VBX_UPD
}

template <int STORAGE>
void warm_update_grids() {
    (void)update_grid<STORAGE, 16, 16, 16, 256>(); (void)update_grid<STORAGE, 16, 16, 8, 256>();
    (void)update_grid<STORAGE, 16, 16, 4, 256>();  (void)update_grid<STORAGE, 8, 16, 16, 256>();
    (void)update_grid<STORAGE, 8, 8, 16, 256>();   (void)update_grid<STORAGE, 4, 8, 16, 256>();
    (void)update_grid<STORAGE, 16, 16, 16, 1024>(); (void)update_grid<STORAGE, 16, 16, 8, 1024>();
    (void)update_grid<STORAGE, 16, 16, 4, 1024>();  (void)update_grid<STORAGE, 16, 16, 8, 512>();
    (void)update_grid<STORAGE, 16, 16, 8, 512, true>(); (void)update_grid<STORAGE, 16, 16, 8, 256, true>();
    (void)update_grid<STORAGE, 16, 16, 4, 256, true>();
}

void launch_update(int storage, int variant, hipStream_t st, const Job* jobs, const MapDesc* maps,
                   const u64* t_key, const int* t_slot, const u32* off, const u32* order, const float4* sorted,
                   u32 JM, u64* touch_key, u32* touch_n, u32 touch_cap, int keep, JobStat* jst, CallState* cs) {
    if (storage == VBX_F32)
        launch_update_s<0>(variant, st, jobs, maps, t_key, t_slot, off, order, sorted, JM, touch_key, touch_n,
                           touch_cap, keep, jst, cs);
    else if (storage == VBX_F16)
        launch_update_s<1>(variant, st, jobs, maps, t_key, t_slot, off, order, sorted, JM, touch_key, touch_n,
                           touch_cap, keep, jst, cs);
    else
        launch_update_s<2>(variant, st, jobs, maps, t_key, t_slot, off, order, sorted, JM, touch_key, touch_n,
                           touch_cap, keep, jst, cs);
}

// Lays a call's scratch buffers out in [base, base + cap), each aligned to 256 bytes.
// VBX_ERR_LIMIT when they do not fit.
int carve_scratch(Scratch* s, char* base, size_t cap, const CallPlan& plan, const ScratchSizes& z, int njobs) {
    size_t off = 0;
    bool fits = true;
    for_each_scratch(s, plan, z, njobs, [&](DevBuf& b, size_t bytes) {
        off = (off + 255) & ~(size_t)255;
        if (bytes == 0) bytes = 256;
        if (!fits || bytes > cap || off > cap - bytes) {
            fits = false;
            return;
        }
        b.p = base + off;
        b.bytes = bytes;
        off += bytes;
    });
    if (!fits) return VBX_ERR_LIMIT;
    note_scratch_sizes(s, z);
    return VBX_OK;
}

// The region's state every call expects to find: an empty block set, zero sort bins, per-frame
// and per-call counters.  Fill kernels only (no memset API).
int clear_carved(Scratch* s, hipStream_t st, int njobs) {
    hipLaunchKernelGGL(k_fill_u64, dim3(grid_for(s->tkey_cap)), dim3(256), 0, st, (u64*)s->tkeys.p, kEmpty,
                       s->tkey_cap);
    hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(s->bins_cap + 1)), dim3(256), 0, st, (u32*)s->bins.p, 0u,
                       s->bins_cap + 1);
    hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(s->hbins_cap)), dim3(256), 0, st, (u32*)s->hbins.p, 0u,
                       s->hbins_cap);
    const size_t jst_words = (size_t)njobs * sizeof(JobStat) / 8;
    hipLaunchKernelGGL(k_fill_u64, dim3(grid_for(jst_words)), dim3(256), 0, st, (u64*)s->jst.p, 0ull, jst_words);
    hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(256), 0, st, (u32*)s->cs.p, 0u, sizeof(CallState) / 4);
    return hipGetLastError() == hipSuccess ? VBX_OK : VBX_ERR_DEVICE;
}


// Records the start / end of a stage on the stream when profiling is on.
struct StageTimer {
    vbx_map* m;
    hipStream_t st;
    int stage;
    hipEvent_t a = nullptr;
    StageTimer(vbx_map* m_, hipStream_t s_, int stage_) : m(m_), st(s_), stage(stage_) {
        if (m && ((m->prof.mask >> stage) & 1u) && (a = m->prof.take())) (void)hipEventRecord(a, st);
    }
    ~StageTimer() {
        if (!a) return;
        hipEvent_t b = m->prof.take();
        if (!b) {
            m->prof.spare.push_back(a);
            return;
        }
        (void)hipEventRecord(b, st);
        m->prof.pending.push_back({stage, a, b});
    }
};

// Host description of one integration call: the launch plan and the map and job tables.
struct Prepared {
    CallPlan plan;
    std::vector<Job> jobs;
    std::vector<MapDesc> descs;
    size_t sum_capacity = 0;
};

// Validates the frames of a call over `maps` (frames[i] belongs to maps[owner[i]]; frames of one
// map are in call order) and numbers the tiles of every frame over the whole call.
int prepare_call(const std::vector<vbx_map*>& maps, const std::vector<vbx_frame>& frames,
                 const std::vector<int>& owner, Prepared& out, const Intrinsics* projective = nullptr) {
    vbx_map* lead = maps[0];
    const int M = (int)maps.size();
    const int F = (int)frames.size();
    if (F > VBX_MAX_FRAMES_PER_CALL) return VBX_ERR_LIMIT;
    std::vector<std::vector<int>> per_map(M);
    for (int i = 0; i < F; ++i) per_map[owner[i]].push_back(i);
    CallPlan& plan = out.plan;
    plan = CallPlan();
    plan.storage = lead->P.storage;
    out.sum_capacity = 0;
    for (int m = 0; m < M; ++m) {
        const vbx_map_params& P = maps[m]->P;
        if (P.storage != plan.storage) return VBX_ERR_INVALID_ARG;
        if (P.merge != lead->P.merge) return VBX_ERR_INVALID_ARG;
        plan.JM = std::max<int>(plan.JM, (int)per_map[m].size());
        plan.max_blocks = std::max(plan.max_blocks, max_blocks_per_ray(P));
        plan.max_vox = std::max(plan.max_vox, max_voxels_per_ray(P));
        plan.keep_touches = plan.keep_touches || (P.flags & VBX_FLAG_KEEP_TOUCHES);
        plan.color = plan.color || (!projective && (P.flags & VBX_FLAG_COLOR));
        out.sum_capacity += maps[m]->capacity;
    }
    plan.grouped = lead->P.merge == VBX_MERGE_GROUPED;
    if (projective) {
        // the blocks come from every point's band (no grouping); the voxels are projected
        plan.grouped = false;
        plan.projective = true;
        plan.K = *projective;
    }

    std::vector<Job>& jobs = out.jobs;
    std::vector<MapDesc>& descs = out.descs;
    jobs.clear();
    descs.clear();
    jobs.reserve(F);
    for (int m = 0; m < M; ++m) {
        descs.push_back(make_desc(maps[m], m, (int)jobs.size(), (int)per_map[m].size()));
        for (size_t k = 0; k < per_map[m].size(); ++k) {
            const vbx_frame& fr = frames[per_map[m][k]];
            Job j;
            std::memset(&j, 0, sizeof j);
            if (fr.n > VBX_MAX_POINTS_PER_FRAME) return VBX_ERR_LIMIT;
            if (fr.n > 0 && !fr.points) return VBX_ERR_INVALID_ARG;
            if (fr.width > 0 && fr.n % fr.width != 0) return VBX_ERR_INVALID_ARG;
            for (int q = 0; q < 12; ++q)
                if (!std::isfinite(fr.pose[q])) return VBX_ERR_INVALID_ARG;
            // a colour map's raycasting frames carry a colour per point
            if (plan.color && (maps[m]->P.flags & VBX_FLAG_COLOR) && fr.n > 0 && !fr.colors)
                return VBX_ERR_INVALID_ARG;
            j.pts = fr.points;
            j.colors = plan.color ? fr.colors : nullptr;
            j.n = (u32)fr.n;
            j.width = fr.width;
            j.map = (u32)m;
            j.jm = (u32)k;
            std::memcpy(j.pose, fr.pose, sizeof j.pose);
            jobs.push_back(j);
            plan.total_points += fr.n;
        }
    }
    u32 total_tiles = 0;
    for (Job& j : jobs) {
        u32 nt;
        if (!plan.grouped) {
            nt = (j.n + kTileSimple - 1) / kTileSimple;
        } else if (j.width > 0) {
            const u32 rows = j.n / j.width;
            nt = ((j.width + kTileGroupedW - 1) / kTileGroupedW) * ((rows + kTileGroupedH - 1) / kTileGroupedH);
        } else {
            nt = (j.n + kTileGrouped - 1) / kTileGrouped;
        }
        j.tile0 = total_tiles;
        j.ntiles = nt;
        total_tiles += nt;
    }
    plan.tiles = total_tiles;
    plan.ray_slots = (size_t)total_tiles * (plan.grouped ? kTileGrouped : kTileSimple);
    plan.tiles_per_job = 0;
    if (M == 1 && !jobs.empty() && jobs[0].ntiles > 0) {
        bool uniform = true;
        for (const Job& j : jobs) uniform = uniform && j.ntiles == jobs[0].ntiles;
        if (uniform) plan.tiles_per_job = jobs[0].ntiles;
    }
    return VBX_OK;
}

// Copies the map and job tables to the device through the pinned staging ring.
int stage_tables(Scratch* s, hipStream_t st, const Prepared& pr) {
    Stage& sg = s->stage[s->stage_i];
    s->stage_i = (s->stage_i + 1) % 4;
    if (sg.used) VBX_TRY(hipEventSynchronize(sg.ev));
    const size_t map_bytes = pr.descs.size() * sizeof(MapDesc);
    const size_t job_bytes = pr.jobs.size() * sizeof(Job);
    if (map_bytes + job_bytes > s->tables.bytes) return VBX_ERR_INVALID_ARG;
    if (sg.bytes < map_bytes + job_bytes) {
        if (sg.host) (void)hipHostFree(sg.host);
        sg.host = nullptr;
        sg.bytes = 0;
        if (hipHostMalloc(&sg.host, map_bytes + job_bytes, hipHostMallocDefault) != hipSuccess) {
            sg.host = nullptr;
            return VBX_ERR_OUT_OF_MEMORY;
        }
        sg.bytes = map_bytes + job_bytes;
    }
    if (!sg.ev && hipEventCreateWithFlags(&sg.ev, hipEventDisableTiming) != hipSuccess) return VBX_ERR_DEVICE;
    std::memcpy(sg.host, pr.descs.data(), map_bytes);
    std::memcpy((char*)sg.host + map_bytes, pr.jobs.data(), job_bytes);
    VBX_TRY(hipMemcpyAsync(s->tables.p, sg.host, map_bytes + job_bytes, hipMemcpyHostToDevice, st));
    VBX_TRY(hipEventRecord(sg.ev, st));
    sg.used = true;
    return VBX_OK;
}

// Copies the map and job tables into s->tables through the arguments of word-copy launches.
int put_tables(Scratch* s, hipStream_t st, const Prepared& pr) {
    const size_t map_bytes = pr.descs.size() * sizeof(MapDesc);
    const size_t job_bytes = pr.jobs.size() * sizeof(Job);
    static_assert(sizeof(MapDesc) % 4 == 0 && sizeof(Job) % 4 == 0, "tables are whole words");
    if (map_bytes + job_bytes > s->tables.bytes) return VBX_ERR_INVALID_ARG;
    const unsigned char* src[2] = {(const unsigned char*)pr.descs.data(), (const unsigned char*)pr.jobs.data()};
    const size_t len[2] = {map_bytes, job_bytes};
    size_t dst_off = 0;
    for (int part = 0; part < 2; ++part) {
        for (size_t o = 0; o < len[part]; o += sizeof(TableChunk)) {
            const size_t n = std::min(sizeof(TableChunk), len[part] - o);
            TableChunk c;
            std::memcpy(c.w, src[part] + o, n);
            hipLaunchKernelGGL(k_put_words, dim3(1), dim3(256), 0, st, c, (u32)(n / 4),
                               (u32*)((char*)s->tables.p + dst_off));
            dst_off += n;
        }
    }
    return hipGetLastError() == hipSuccess ? VBX_OK : VBX_ERR_DEVICE;
}

// Per device: the region's device address (from hipGetSymbolAddress, with that device current,
// once) and the host description of the buffers laid out in it.
struct NoAllocDevice {
    std::once_flag once;
    hipError_t status = hipSuccess;
    void* ptr = nullptr;
    std::mutex lock;   // the host-side layout below is rewritten by every call
    Scratch layout;
};
constexpr int kNoAllocDevices = 64;
NoAllocDevice g_noalloc[kNoAllocDevices];

// Resolves the once-per-process launch shapes before any capture.
void warm_launch_shapes() {
    (void)group_merge_grid();
    (void)sort_resident_waves();
    (void)cross_grid();
    warm_update_grids<0>();
    warm_update_grids<1>();
    warm_update_grids<2>();
}

// The kernel sequence of one call over the staged tables in `s`.  Only kernel launches are
// made here (no copies, fills through the memset API, allocations or host waits), so the
// sequence can be captured into a graph.  `timer` is the map whose profiler records the
// stages, or null.
int launch_call(Scratch* s, hipStream_t st, const CallPlan& plan, int J, int M, int update_variant,
                vbx_map* timer) {
    vbx_map* prof_map = timer;
    const size_t map_bytes = (size_t)M * sizeof(MapDesc);
    const MapDesc* d_maps = (const MapDesc*)s->tables.p;
    const Job* d_jobs = (const Job*)((char*)s->tables.p + map_bytes);
    CallState* cs = (CallState*)s->cs.p;
    JobStat* jst = (JobStat*)s->jst.p;
    float4* rays_p = (float4*)s->rays_p.p;
    u32* rays_job = (u32*)s->rays_job.p;
    u32* rays_c = plan.color ? (u32*)s->rays_c.p : nullptr;
    u32* sorted_c = plan.color ? (u32*)s->sorted_c.p : nullptr;
    const PartialColor* parts_c = plan.color ? (const PartialColor*)s->parts_c.p : nullptr;
    PartialColor* parts_sorted_c = plan.color ? (PartialColor*)s->parts_sorted_c.p : nullptr;
    const u32 ray_cap = (u32)s->ray_cap;
    const u32 total_tiles = plan.tiles;

    const u32 JM = (u32)plan.JM;
    const unsigned GT = grid_for(s->tlist_cap, 1024);
    const unsigned NP = (unsigned)std::max<size_t>(s->nparts, 1);
    // exclusive scan of the t_count * per_block bin counts
    auto scan_bins = [&](u32 per_block, u32* chunk_first, u32* hsrc) {
        hipLaunchKernelGGL(k_scan_sums, dim3(NP), dim3(256), 0, st, (u32*)s->bins.p, per_block,
                           (u32*)s->partial.p, (u32*)s->off.p, cs, hsrc, (const u32*)s->tlist.p,
                           (u32)s->tlist_cap);
        hipLaunchKernelGGL(k_scan_final, dim3(NP), dim3(256), 0, st, (const u32*)s->bins.p, (const u32*)s->partial.p,
                           (u32*)s->off.p, per_block, chunk_first, (const CallState*)cs);
    };
    const u32 JMS = JM * (u32)kGroupSubBins;   // partial-group sort bins per block
    // points
    if (total_tiles > 0) {
        StageTimer tm(prof_map, st, ST_POINTS);
        if (!plan.grouped) {
            hipLaunchKernelGGL(k_points_simple, dim3(total_tiles), dim3(256), 0, st, d_jobs, J, d_maps, rays_p,
                               rays_job, rays_c, jst, cs);
        } else if (!plan.color) {
            hipLaunchKernelGGL(k_points_grouped<false>, dim3(total_tiles), dim3(256), 0, st, d_jobs, J, d_maps,
                               (u64*)s->tkeys.p, (u32)(s->tkey_cap - 1), (u32*)s->tlist.p, (u32)s->tlist_cap,
                               (Partial*)s->parts.p, (PartialColor*)nullptr, (u32*)s->tile_parts.p,
                               plan.tiles_per_job, jst, cs);
        } else {
            hipLaunchKernelGGL(k_points_grouped<true>, dim3(total_tiles), dim3(256), 0, st, d_jobs, J, d_maps,
                               (u64*)s->tkeys.p, (u32)(s->tkey_cap - 1), (u32*)s->tlist.p, (u32)s->tlist_cap,
                               (Partial*)s->parts.p, (PartialColor*)s->parts_c.p, (u32*)s->tile_parts.p,
                               plan.tiles_per_job, jst, cs);
        }
    }
    if (plan.grouped && total_tiles > 0) {
        StageTimer tm(prof_map, st, ST_GROUPS);
        // two tiles per wave once the paired waves still fill the chip twice over
        const u32 tpw = total_tiles >= 4u * sort_resident_waves() ? 2u : 1u;
        const unsigned GW = (total_tiles + 4 * tpw - 1) / (4 * tpw);
        hipLaunchKernelGGL(k_densify, dim3(GT), dim3(256), 0, st, (const u32*)s->tlist.p, (u32)s->tlist_cap,
                           (u32*)s->tval.p, (const CallState*)cs);
        hipLaunchKernelGGL(k_gbin_count, dim3(GW), dim3(256), 0, st, (const Partial*)s->parts.p,
                           (const u32*)s->tile_parts.p, total_tiles, (const u32*)s->tval.p, (u32*)s->bins.p, JM,
                           tpw, (const CallState*)cs);
        scan_bins(JMS, (u32*)s->chunk_first.p, nullptr);
        hipLaunchKernelGGL(k_gscatter, dim3(GW), dim3(256), 0, st, (const Partial*)s->parts.p,
                           (const u32*)s->tile_parts.p, total_tiles, (const u32*)s->tval.p, (u32*)s->bins.p,
                           (const u32*)s->off.p, JM, tpw, (Partial*)s->parts_sorted.p, parts_c, parts_sorted_c,
                           (const CallState*)cs);
        if (!plan.color)
            hipLaunchKernelGGL(k_group_merge<false>, dim3(group_merge_grid()), dim3(256), 0, st, d_jobs, d_maps,
                               (const u64*)s->tkeys.p, (const u32*)s->tlist.p, (const u32*)s->off.p,
                               (const u32*)s->chunk_first.p, (const Partial*)s->parts_sorted.p, JMS,
                               (const PartialColor*)nullptr, rays_p, rays_job, (u32*)nullptr, jst, cs);
        else
            hipLaunchKernelGGL(k_group_merge<true>, dim3(group_merge_grid()), dim3(256), 0, st, d_jobs, d_maps,
                               (const u64*)s->tkeys.p, (const u32*)s->tlist.p, (const u32*)s->off.p,
                               (const u32*)s->chunk_first.p, (const Partial*)s->parts_sorted.p, JMS,
                               (const PartialColor*)parts_sorted_c, rays_p, rays_job, rays_c, jst, cs);
    }
    const unsigned G = grid_for(plan.ray_slots, 2048);
    const unsigned GC = std::min(G, cross_grid());
    const u32 MB = (u32)plan.max_blocks;
    {
    StageTimer tm(prof_map, st, ST_CROSS);
    // raycasting calls count their crossings here (by block-set slot and frame); projection
    // mapping counts them in its own pass
    hipLaunchKernelGGL(k_cross, dim3(GC), dim3(256), 0, st, d_jobs, d_maps, (const float4*)rays_p,
                       (const u32*)rays_job, (u64*)s->tkeys.p, (u32)(s->tkey_cap - 1), (u32*)s->tlist.p,
                       (u32)s->tlist_cap, (u32*)s->cross.p, (unsigned char*)s->ncross.p, MB,
                       plan.projective ? (u32*)nullptr : (u32*)s->hbins.p, JM, jst, cs, ray_cap);
    }
    {
    StageTimer tm(prof_map, st, ST_RESOLVE);
    hipLaunchKernelGGL(k_resolve, dim3(GT), dim3(256), 0, st, d_maps, (const u64*)s->tkeys.p, (u32*)s->tval.p,
                       (const u32*)s->tlist.p, (u64*)s->t_key.p, (int*)s->t_slot.p, cs);
    }
    {
    StageTimer tm(prof_map, st, ST_COMMIT);
    hipLaunchKernelGGL(k_commit, dim3(GT), dim3(256), 0, st, d_maps, (const u64*)s->t_key.p, (int*)s->t_slot.p, cs);
    }
    if (plan.projective) {
        {
        StageTimer tm(prof_map, st, ST_BINS);
        // which frames' bands cross which blocks: the crossing counts per (block, frame)
        hipLaunchKernelGGL(k_bin_count, dim3(G), dim3(256), 0, st, d_jobs, (const u32*)s->cross.p,
                           (const unsigned char*)s->ncross.p, MB, (const u32*)s->tval.p, (const u32*)rays_job,
                           (u32*)s->bins.p, JM, cs, ray_cap);
        }
        if (plan.keep_touches) hipLaunchKernelGGL(k_set_u32, dim3(1), dim3(1), 0, st, &cs->touch_count, 0u);
        StageTimer tm(prof_map, st, ST_UPDATE);
        const unsigned GP = 2048;   // persistent: workgroups stride over the call's blocks
#define VBX_PROJ(S)                                                                                           \
        hipLaunchKernelGGL(k_project<S>, dim3(GP), dim3(256), 0, st, d_jobs, d_maps, (const u64*)s->t_key.p,   \
                           (const int*)s->t_slot.p, (u32*)s->bins.p, JM, plan.K, (u64*)s->touch_key.p,          \
                           (u32*)s->touch_n.p,                                                                 \
                           (u32)s->touch_cap, plan.keep_touches ? 1 : 0, jst, cs)
        if (plan.storage == VBX_F32) VBX_PROJ(0);
        else if (plan.storage == VBX_F16) VBX_PROJ(1);
        else VBX_PROJ(2);
#undef VBX_PROJ
    } else {
    {
    // the counts by (block, frame), gathered from the crossing kernel's counts by block-set slot
    StageTimer tm(prof_map, st, ST_SCAN);
    scan_bins(JM, nullptr, (u32*)s->hbins.p);
    }
    {
    StageTimer tm(prof_map, st, ST_SCATTER);
    hipLaunchKernelGGL(k_scatter, dim3(G), dim3(256), 0, st, d_jobs, (const u32*)s->cross.p,
                       (const unsigned char*)s->ncross.p, MB, (const u32*)s->tval.p, (const u32*)rays_job,
                       (u32*)s->bins.p, (const u32*)s->off.p, JM, (const float4*)rays_p, (float4*)s->sorted.p,
                       (const u32*)rays_c, sorted_c, cs, ray_cap);
    }
    if (plan.keep_touches) hipLaunchKernelGGL(k_set_u32, dim3(1), dim3(1), 0, st, &cs->touch_count, 0u);
    {
    StageTimer tm(prof_map, st, ST_UPDATE);
    hipLaunchKernelGGL(k_order_blocks, dim3(1), dim3(1024), 0, st, (const u32*)s->off.p, JM, (u32*)s->order.p,
                       (const CallState*)cs);
    if (!plan.color) {
        launch_update(plan.storage, update_variant, st, d_jobs, d_maps, (const u64*)s->t_key.p,
                      (const int*)s->t_slot.p, (const u32*)s->off.p, (const u32*)s->order.p,
                      (const float4*)s->sorted.p, JM,
                      (u64*)s->touch_key.p, (u32*)s->touch_n.p, (u32)s->touch_cap, plan.keep_touches ? 1 : 0,
                      jst, cs);
    } else {
        // colour calls: z-slab regions, one frame per step, the colour sums beside the others.
        // The candidates whose sums fit the LDS: quarter blocks of 256 threads (the default;
        // 0.56 ms on the 100-frame room against 0.66 for half blocks of 512 threads and 0.87 for
        // half blocks of 256), chosen by the (2, 0, 256) and (2, 0, 512) tunings otherwise.
#define VBX_UPD_COLOR(S, Z, T)                                                                               \
        launch_update_t<S, 16, 16, Z, T, true>(st, d_jobs, d_maps, (const u64*)s->t_key.p,                    \
                                               (const int*)s->t_slot.p, (const u32*)s->off.p,                  \
                                               (const u32*)s->order.p, (const float4*)s->sorted.p,             \
                                               (const u32*)sorted_c, JM, (u64*)s->touch_key.p,                 \
                                               (u32*)s->touch_n.p, (u32)s->touch_cap,                          \
                                               plan.keep_touches ? 1 : 0, jst, cs)
#define VBX_UPD_COLOR_S(S)                                                                                   \
        if (update_variant == 1) VBX_UPD_COLOR(S, 8, 256);                                                    \
        else if (update_variant == 9) VBX_UPD_COLOR(S, 8, 512);                                               \
        else VBX_UPD_COLOR(S, 4, 256)
        if (plan.storage == VBX_F32) { VBX_UPD_COLOR_S(0); }
        else if (plan.storage == VBX_F16) { VBX_UPD_COLOR_S(1); }
        else { VBX_UPD_COLOR_S(2); }
#undef VBX_UPD_COLOR_S
#undef VBX_UPD_COLOR
    }
    }
    }
    {
    StageTimer tm(prof_map, st, ST_FINISH);
    // one workgroup per map, and few for the block-set cleanup: every workgroup adds to one
    // completion counter, and such adds are carried out one after another
    hipLaunchKernelGGL(k_finish_call, dim3(M + grid_for(s->tkey_cap, 32)), dim3(256), 0, st, d_jobs, d_maps, M,
                       jst, (u64*)s->tkeys.p, (u32)s->tkey_cap, (const u32*)s->tlist.p, (u32)s->tlist_cap, cs);
    }
    if (hipGetLastError() != hipSuccess) return VBX_ERR_DEVICE;
    return VBX_OK;
}

// Records which scratch holds the touches of the maps of the last call.
void note_touches(Scratch* s, const std::vector<vbx_map*>& maps, const CallPlan& plan) {
    if (!plan.keep_touches) return;
    s->last_maps = maps;
    s->touches_valid = true;
    for (size_t m = 0; m < maps.size(); ++m) {
        maps[m]->touch_src = s;
        maps[m]->touch_idx = (int)m;
    }
}

// One integration call over `maps` (distinct maps) with frames[i] belonging to
// maps[owner[i]]; frames of one map are in call order.  Runs on stream `st` with scratch `s`.
int run_call_on(Scratch* s, hipStream_t st, std::vector<vbx_map*>& maps, const std::vector<vbx_frame>& frames,
                const std::vector<int>& owner, int update_variant, vbx_map* timer,
                const Intrinsics* projective = nullptr) {
    if (frames.empty()) return VBX_OK;
    Prepared pr;
    int rc = prepare_call(maps, frames, owner, pr, projective);
    if (rc != VBX_OK) return rc;
    const int J = (int)pr.jobs.size(), M = (int)maps.size();
    if ((rc = ensure_scratch(s, st, pr.plan, J, M, pr.sum_capacity)) != VBX_OK) return rc;
    if ((rc = stage_tables(s, st, pr)) != VBX_OK) return rc;
    if ((rc = launch_call(s, st, pr.plan, J, M, update_variant, timer)) != VBX_OK) return rc;
    note_touches(s, maps, pr.plan);
    return VBX_OK;
}

// A call on maps[0]'s scratch and stream.
int run_call(std::vector<vbx_map*>& maps, const std::vector<vbx_frame>& frames,
             const std::vector<int>& owner) {
    vbx_map* lead = maps[0];
    return run_call_on(lead->scratch, lead->stream, maps, frames, owner, lead->update_variant, lead);
}

// Device memory a map of `capacity` blocks holds (hash table, block pool, state).
uint64_t map_storage_bytes(const vbx_map_params& P, uint64_t capacity) {
    const uint64_t hcap = next_pow2((size_t)capacity * 2);
    const uint64_t vb = P.storage == VBX_F32 ? 8 : 4;
    return hcap * (sizeof(u64) + sizeof(int)) + capacity * 4096 * vb + sizeof(MapState);
}

int read_state(vbx_map* m, MapState* out) {
    VBX_TRY(hipStreamSynchronize(m->stream));
    VBX_TRY(hipMemcpy(out, m->st, sizeof(MapState), hipMemcpyDeviceToHost));
    return VBX_OK;
}

// Host-side insertion with the device's probe order (linear probing from mix64(key)).
void host_insert(std::vector<u64>& keys, std::vector<int>& slots, u64 key, int slot) {
    const u32 mask = (u32)keys.size() - 1;
    u32 h = (u32)mix64(key) & mask;
    while (keys[h] != kEmpty && keys[h] != key) h = (h + 1) & mask;
    keys[h] = key;
    slots[h] = slot;
}

// One block of host values (dw [4096][2]: D metres, W) in the map's pool format.
void encode_block(const vbx_map* m, const float* dw, unsigned char* out) {
    for (int l = 0; l < 4096; ++l) {
        const float D = dw[2 * l];
        const float W = dw[2 * l + 1];
        if (m->P.storage == VBX_F32) {
            float* v = (float*)out + 2 * l;
            v[0] = D;
            v[1] = W;
        } else {
            const float dn = D / m->P.trunc;
            const uint32_t dc = m->P.storage == VBX_F16 ? (uint32_t)__half_as_ushort(__float2half_rn(dn))
                                                        : (uint32_t)s16_encode(dn);
            const uint32_t wc = __half_as_ushort(__float2half_rn(W));
            ((uint32_t*)out)[l] = dc | (wc << 16);
        }
    }
}

// ---- ESDF layer (host side) ------------------------------------------------------------

// Grows the layer's voxel words to cover `blocks` pool slots (content kept, new words zero:
// unobserved).
int esdf_grow_vox(vbx_map* m, size_t blocks) {
    Esdf* e = m->esdf;
    if (blocks <= e->vox_blocks) return VBX_OK;
    u64* nv = nullptr;
    if (map_alloc(m, (void**)&nv, blocks * 4096 * sizeof(u64)) != VBX_OK) return VBX_ERR_OUT_OF_MEMORY;
    if (e->vox_blocks)
        VBX_TRY(hipMemcpyAsync(nv, e->vox, e->vox_blocks * 4096 * sizeof(u64), hipMemcpyDeviceToDevice, m->stream));
    const size_t fresh = (blocks - e->vox_blocks) * 4096;
    hipLaunchKernelGGL(k_fill_u64, dim3(grid_for(fresh)), dim3(256), 0, m->stream, nv + e->vox_blocks * 4096, 0ull,
                       fresh);
    VBX_TRY(hipStreamSynchronize(m->stream));
    map_free(m, e->vox);
    e->vox = nv;
    e->vox_blocks = blocks;
    return VBX_OK;
}

// Grows the dirty flags to the pool capacity (flags kept, new ones clear).
int esdf_grow_dirty(vbx_map* m) {
    Esdf* e = m->esdf;
    if (m->capacity <= e->dirty_cap) return VBX_OK;
    u32* nd = nullptr;
    if (map_alloc(m, (void**)&nd, (size_t)m->capacity * sizeof(u32)) != VBX_OK) return VBX_ERR_OUT_OF_MEMORY;
    hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(m->capacity)), dim3(256), 0, m->stream, nd, 0u, (size_t)m->capacity);
    if (e->dirty_cap)
        VBX_TRY(hipMemcpyAsync(nd, e->dirty, (size_t)e->dirty_cap * sizeof(u32), hipMemcpyDeviceToDevice, m->stream));
    VBX_TRY(hipStreamSynchronize(m->stream));
    map_free(m, e->dirty);
    e->dirty = nd;
    e->dirty_cap = m->capacity;
    return VBX_OK;
}

// Every voxel unobserved and the first `mark` pool slots dirty (after the map was cleared or
// replaced).
void esdf_reset(vbx_map* m, size_t mark) {
    Esdf* e = m->esdf;
    if (!e) return;
    e->nbr_blocks = 0;   // the blocks were dropped or replaced
    if (e->vox_blocks)
        hipLaunchKernelGGL(k_fill_u64, dim3(grid_for(e->vox_blocks * 4096)), dim3(256), 0, m->stream, e->vox, 0ull,
                           e->vox_blocks * 4096);
    if (e->dirty_cap)
        hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(e->dirty_cap)), dim3(256), 0, m->stream, e->dirty, 0u,
                           (size_t)e->dirty_cap);
    if (mark)
        hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(mark)), dim3(256), 0, m->stream, e->dirty, 1u, mark);
}

void esdf_free(vbx_map* m) {
    Esdf* e = m->esdf;
    if (!e) return;
    map_free(m, e->vox);
    map_free(m, e->dirty);
    DevBuf* bufs[] = {&e->rstamp, &e->lstamp, &e->list, &e->nbr, &e->slot_key, &e->raise0, &e->raise1,
                      &e->lower0, &e->lower1, &e->cnt};
    for (DevBuf* b : bufs)
        if (b->p) (void)hipFree(b->p);
    delete e;
    m->esdf = nullptr;
}

}  // namespace

// ===========================================================================
// Map server: integration requests of many maps batched into ticks as they arrive
// ===========================================================================
namespace {

double server_clock() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

constexpr int kServerSlots = 4;          // status slots; more than the ticks ever in flight
constexpr int kServerMaxMapsPerTick = 127;

struct ServerEntry {
    vbx_sched::Request req;
    vbx_frame frame;
};

struct TickRec {
    std::vector<vbx_sched::Request*> reqs;
    std::vector<int> owner;              // map of each request within the call
    hipEvent_t ev = nullptr;
    int slot = 0;
    int launch_status = VBX_OK;          // a call that could not be launched
};

}  // namespace

struct vbx_server {
    vbx_server_params P;
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    Scratch* scratch = nullptr;
    vbx_sched::Planner planner{0};
    std::vector<vbx_map*> maps;
    std::deque<ServerEntry> entries;     // by ticket - 1
    std::mutex mu;
    std::condition_variable cv_engine, cv_complete, cv_done;
    std::deque<TickRec> inflight;
    std::vector<hipEvent_t> spare_events;
    int* status_dev = nullptr;           // [kServerSlots][128]
    int* status_host = nullptr;          // pinned mirror
    int next_slot = 0;
    std::thread engine, completer;
    bool stop = false;
    // statistics
    uint64_t submitted = 0, finished = 0, failed = 0, ticks = 0, frames = 0, points = 0, replays = 0;
    uint32_t rejected_maps = 0;
    double first_arrival = 1e300, last_done = 0.0;
    std::vector<double> latency;         // seconds, completed requests
};

namespace {

// Finished requests enter the statistics; caller holds the lock.
void server_account(vbx_server* S, const std::vector<vbx_sched::Request*>& fin) {
    for (vbx_sched::Request* r : fin) {
        S->finished++;
        if (r->status != VBX_OK) {
            S->failed++;
            continue;
        }
        S->points += r->points;
        S->latency.push_back(r->t_done - r->t_arrival);
        S->first_arrival = std::min(S->first_arrival, r->t_arrival);
        S->last_done = std::max(S->last_done, r->t_done);
    }
}

// A map whose pool filled: grow it within the budget and queue its turned-away requests
// again; if it cannot grow, clear its error and run them again one at a time, so that only
// a request that overflows the pool on its own fails.  Called with the lock held (released
// around the device calls); the map has no tick in flight.
void server_recover(vbx_server* S, int id, std::unique_lock<std::mutex>& lk) {
    vbx_map* m = S->maps[(size_t)id];
    const size_t n_replay = S->planner.map(id).replay.size();
    const uint64_t cap = m->capacity;
    const uint64_t ncap = cap * 2;
    const uint64_t extra = map_storage_bytes(m->P, ncap) - map_storage_bytes(m->P, cap);
    const bool charged = n_replay > 0 && S->P.grow && ncap <= (1u << 29) && S->planner.grow(id, extra);
    lk.unlock();
    int rc = charged ? vbx_map_reserve(m, (uint32_t)ncap) : VBX_ERR_POOL_FULL;
    if (rc != VBX_OK) (void)vbx_map_clear_error(m);   // the map is as it was before the full call
    lk.lock();
    if (charged && rc != VBX_OK) S->planner.release(id, extra);
    S->replays += n_replay;
    S->planner.requeue(id, rc != VBX_OK);
}

void server_engine(vbx_server* S) {
    (void)hipSetDevice(S->device);
    std::unique_lock<std::mutex> lk(S->mu);
    for (;;) {
        S->cv_engine.wait(lk, [&] {
            return S->stop || ((int)S->inflight.size() < S->P.max_inflight &&
                               (S->planner.has_work() || !S->planner.recoverable().empty()));
        });
        if (S->stop) break;
        const std::vector<int> rec = S->planner.recoverable();
        if (!rec.empty()) {
            server_recover(S, rec[0], lk);
            continue;
        }
        std::vector<vbx_sched::Request*> tick = S->planner.next_tick(
            S->P.max_frames_per_tick, S->P.max_points_per_tick, kServerMaxMapsPerTick);
        if (tick.empty()) {
            // not expected (has_work promises a request); never spin holding the lock
            S->cv_engine.wait_for(lk, std::chrono::milliseconds(1));
            continue;
        }
        // maps of the call in order of first appearance
        std::vector<vbx_map*> cm;
        std::vector<int> ids, owner;
        std::vector<vbx_frame> fr;
        for (const vbx_sched::Request* r : tick) {
            size_t j = 0;
            while (j < ids.size() && ids[j] != r->map) ++j;
            if (j == ids.size()) {
                ids.push_back(r->map);
                cm.push_back(S->maps[(size_t)r->map]);
            }
            owner.push_back((int)j);
            fr.push_back(S->entries[(size_t)(r->ticket - 1)].frame);
        }
        hipEvent_t ev = nullptr;
        if (!S->spare_events.empty()) {
            ev = S->spare_events.back();
            S->spare_events.pop_back();
        }
        const int slot = S->next_slot;
        S->next_slot = (slot + 1) % kServerSlots;
        lk.unlock();
        if (!ev && hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) ev = nullptr;
        int rc = run_call_on(S->scratch, S->stream, cm, fr, owner, cm[0]->update_variant, nullptr);
        if (rc == VBX_OK) {
            hipLaunchKernelGGL(k_map_status, dim3(1), dim3(128), 0, S->stream, (const MapDesc*)S->scratch->tables.p,
                               (int)cm.size(), S->status_dev + 128 * slot);
            if (hipMemcpyAsync(S->status_host + 128 * slot, S->status_dev + 128 * slot, sizeof(int) * cm.size(),
                               hipMemcpyDeviceToHost, S->stream) != hipSuccess)
                rc = VBX_ERR_DEVICE;
        }
        if (!ev || hipEventRecord(ev, S->stream) != hipSuccess) rc = VBX_ERR_DEVICE;
        lk.lock();
        TickRec t;
        t.reqs = std::move(tick);
        t.owner = std::move(owner);
        t.ev = ev;
        t.slot = slot;
        t.launch_status = rc;
        S->ticks++;
        S->frames += t.reqs.size();
        S->inflight.push_back(std::move(t));
        S->cv_complete.notify_one();
    }
}

void server_completer(vbx_server* S) {
    (void)hipSetDevice(S->device);
    std::unique_lock<std::mutex> lk(S->mu);
    for (;;) {
        S->cv_complete.wait(lk, [&] { return S->stop || !S->inflight.empty(); });
        if (S->inflight.empty()) {
            if (S->stop) break;
            continue;
        }
        hipEvent_t ev = S->inflight.front().ev;
        lk.unlock();
        const hipError_t e = ev ? hipEventSynchronize(ev) : hipErrorInvalidValue;
        const double now = server_clock();
        lk.lock();
        TickRec t = std::move(S->inflight.front());
        S->inflight.pop_front();
        std::vector<int> st(t.reqs.size());
        for (size_t i = 0; i < t.reqs.size(); ++i) {
            if (t.launch_status != VBX_OK) st[i] = t.launch_status;
            else if (e != hipSuccess) st[i] = VBX_ERR_DEVICE;
            else st[i] = S->status_host[128 * t.slot + t.owner[i]];
        }
        std::vector<vbx_sched::Request*> fin;
        S->planner.complete(t.reqs, st, now, &fin);
        server_account(S, fin);
        if (ev) S->spare_events.push_back(ev);
        S->cv_engine.notify_one();
        S->cv_done.notify_all();
    }
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

void vbx_default_params(vbx_map_params* p) {
    if (!p) return;
    std::memset(p, 0, sizeof *p);
    p->voxel_size = 0.1f;
    p->trunc = 0.3f;
    p->w_max = 1e4f;
    p->max_range = 5.0f;
    p->z_min = 0.1f;
    p->weighting = VBX_W_CONST;
    p->merge = VBX_MERGE_NONE;
    p->storage = VBX_F32;
    p->dist = VBX_DIST_EQ1;
    p->block_capacity = 65536;
    p->flags = 0;
    p->stream = nullptr;
}

int vbx_map_create_ex(const vbx_map_params* params, vbx_map** out) {
    if (!params || !out) return VBX_ERR_INVALID_ARG;
    int rc = validate_params(*params);
    if (rc != VBX_OK) return rc;
    vbx_map* m = new (std::nothrow) vbx_map();
    if (!m) return VBX_ERR_OUT_OF_MEMORY;
    m->P = *params;
    m->stream = (hipStream_t)params->stream;
    m->voxel_bytes = params->storage == VBX_F32 ? 8 : 4;
    m->wbits = weight_bits(m->P);
    m->kw = sum_bits(m->P);
    m->scratch = new (std::nothrow) Scratch();
    if (const char* e = std::getenv("VBX_UPDATE_VARIANT")) {
        const int v = std::atoi(e);
        if (v >= 0 && v < kNumUpdateVariants) m->update_variant = v;
    }
    // the map's first device allocation comes before any other device call, so a failing
    // allocator hook ends the call without touching the device
    if (!m->scratch || map_alloc(m, (void**)&m->st, sizeof(MapState)) != VBX_OK) {
        delete m->scratch;
        delete m;
        return VBX_ERR_OUT_OF_MEMORY;
    }
    (void)hipGetDevice(&m->device);
    MapState zero;
    std::memset(&zero, 0, sizeof zero);
    if (hipMemcpy(m->st, &zero, sizeof zero, hipMemcpyHostToDevice) != hipSuccess ||
        (rc = alloc_storage(m, params->block_capacity)) != VBX_OK ||
        hipStreamSynchronize(m->stream) != hipSuccess) {
        free_storage(m);
        map_free(m, m->st);
        free_scratch(m->scratch);
        delete m;
        return rc != VBX_OK ? rc : VBX_ERR_DEVICE;
    }
    *out = m;
    return VBX_OK;
}

int vbx_map_create(float voxel_size, float trunc, int weighting, vbx_map** out) {
    vbx_map_params p;
    vbx_default_params(&p);
    p.voxel_size = voxel_size;
    p.trunc = trunc;
    p.weighting = weighting;
    return vbx_map_create_ex(&p, out);
}

void vbx_map_destroy(vbx_map* m) {
    if (!m) return;
    (void)hipStreamSynchronize(m->stream);
    for (auto& r : m->prof.pending) {
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    for (hipEvent_t e : m->prof.spare) (void)hipEventDestroy(e);
    esdf_free(m);
    free_storage(m);
    map_free(m, m->st);
    free_scratch(m->scratch);
    delete m;
}

int vbx_map_set_stream(vbx_map* m, void* stream) {
    if (!m) return VBX_ERR_INVALID_ARG;
    (void)hipStreamSynchronize(m->stream);
    m->stream = (hipStream_t)stream;
    m->P.stream = stream;
    return VBX_OK;
}

int vbx_integrate_frames(vbx_map* m, const vbx_frame* frames, int F) {
    if (!m || F < 0 || (F > 0 && !frames)) return VBX_ERR_INVALID_ARG;
    std::vector<vbx_map*> maps{m};
    std::vector<vbx_frame> fr(frames, frames + F);
    std::vector<int> owner(F, 0);
    return run_call(maps, fr, owner);
}

int vbx_integrate_frames_noalloc(vbx_map* m, const vbx_frame* frames, int F) {
    if (!m || F < 0 || (F > 0 && !frames)) return VBX_ERR_INVALID_ARG;
    int dev = -1;
    VBX_TRY(hipGetDevice(&dev));
    if (dev != m->device || dev < 0 || dev >= kNoAllocDevices) return VBX_ERR_INVALID_ARG;
    NoAllocDevice& D = g_noalloc[dev];
    std::call_once(D.once, [&D] { D.status = hipGetSymbolAddress(&D.ptr, HIP_SYMBOL(scratch)); });
    if (D.status != hipSuccess || !D.ptr) return VBX_ERR_DEVICE;
    if (F == 0) return VBX_OK;
    std::vector<vbx_map*> maps{m};
    std::vector<vbx_frame> fr(frames, frames + F);
    std::vector<int> owner(F, 0);
    Prepared pr;
    int rc = prepare_call(maps, fr, owner, pr);
    if (rc != VBX_OK) return rc;
    pr.plan.keep_touches = false;
    const int J = (int)pr.jobs.size();
    ScratchSizes z;
    if ((rc = scratch_sizes(pr.plan, J, 1, pr.sum_capacity, z)) != VBX_OK) return rc;
    std::lock_guard<std::mutex> g(D.lock);
    Scratch* s = &D.layout;
    if ((rc = carve_scratch(s, (char*)D.ptr, VBX_NOALLOC_SCRATCH_BYTES, pr.plan, z, J)) != VBX_OK) return rc;
    hipStream_t st = m->stream;
    if ((rc = clear_carved(s, st, J)) != VBX_OK) return rc;
    if ((rc = put_tables(s, st, pr)) != VBX_OK) return rc;
    if ((rc = launch_call(s, st, pr.plan, J, 1, m->update_variant, nullptr)) != VBX_OK) return rc;
    m->touch_src = nullptr;   // no touch records for this call
    return VBX_OK;
}

int vbx_integrate_projective(vbx_map* m, const vbx_frame* frames, int F, const float intrinsics[4]) {
    if (!m || F < 0 || (F > 0 && (!frames || !intrinsics))) return VBX_ERR_INVALID_ARG;
    if (F == 0) return VBX_OK;
    Intrinsics K{intrinsics[0], intrinsics[1], intrinsics[2], intrinsics[3]};
    if (!(K.fx > 0.0f) || !(K.fy > 0.0f) || !std::isfinite(K.fx) || !std::isfinite(K.fy) || !std::isfinite(K.cx) ||
        !std::isfinite(K.cy))
        return VBX_ERR_INVALID_ARG;
    for (int i = 0; i < F; ++i)
        if (frames[i].width == 0 || frames[i].n % frames[i].width != 0) return VBX_ERR_INVALID_ARG;
    std::vector<vbx_map*> maps{m};
    std::vector<vbx_frame> fr(frames, frames + F);
    std::vector<int> owner(F, 0);
    return run_call_on(m->scratch, m->stream, maps, fr, owner, m->update_variant, m, &K);
}

int vbx_integrate(vbx_map* m, const float* points_dev, size_t n, const float pose[12]) {
    if (!m || !pose || (n > 0 && !points_dev)) return VBX_ERR_INVALID_ARG;
    vbx_frame f;
    std::memset(&f, 0, sizeof f);
    f.points = points_dev;
    f.n = n;
    std::memcpy(f.pose, pose, sizeof f.pose);
    return vbx_integrate_frames(m, &f, 1);
}

int vbx_integrate_batch(vbx_map* m, const float* const* points_dev, const size_t* n,
                        const float* poses, int F) {
    if (!m || F < 0 || (F > 0 && (!points_dev || !n || !poses))) return VBX_ERR_INVALID_ARG;
    std::vector<vbx_frame> fr(F);
    for (int i = 0; i < F; ++i) {
        std::memset(&fr[i], 0, sizeof fr[i]);
        fr[i].points = points_dev[i];
        fr[i].n = n[i];
        std::memcpy(fr[i].pose, poses + 12 * i, sizeof fr[i].pose);
    }
    return vbx_integrate_frames(m, fr.data(), F);
}

int vbx_integrate_multi(vbx_map* const* maps, const vbx_frame* frames, int M) {
    if (!maps || !frames || M <= 0) return VBX_ERR_INVALID_ARG;
    if (M > 127) return VBX_ERR_LIMIT;
    std::vector<vbx_map*> mv(maps, maps + M);
    for (int i = 0; i < M; ++i) {
        if (!mv[i]) return VBX_ERR_INVALID_ARG;
        for (int j = 0; j < i; ++j)
            if (mv[j] == mv[i]) return VBX_ERR_INVALID_ARG;
    }
    std::vector<vbx_frame> fr(frames, frames + M);
    std::vector<int> owner(M);
    for (int i = 0; i < M; ++i) owner[i] = i;
    return run_call(mv, fr, owner);
}

int vbx_map_sync(vbx_map* m) {
    if (!m) return VBX_ERR_INVALID_ARG;
    MapState s;
    int rc = read_state(m, &s);
    if (rc != VBX_OK) return rc;
    return s.error;
}

int vbx_map_clear_error(vbx_map* m) {
    if (!m) return VBX_ERR_INVALID_ARG;
    MapState s;
    int rc = read_state(m, &s);
    if (rc != VBX_OK) return rc;
    s.error = 0;
    VBX_TRY(hipMemcpy(m->st, &s, sizeof s, hipMemcpyHostToDevice));
    return VBX_OK;
}

int vbx_map_num_blocks(vbx_map* m, size_t* n_out) {
    if (!m || !n_out) return VBX_ERR_INVALID_ARG;
    MapState s;
    int rc = read_state(m, &s);
    if (rc != VBX_OK) return rc;
    *n_out = s.block_count;
    return VBX_OK;
}

int vbx_map_reserve(vbx_map* m, uint32_t block_capacity) {
    if (!m || block_capacity == 0 || block_capacity > (1u << 29)) return VBX_ERR_INVALID_ARG;
    MapState s;
    int rc = read_state(m, &s);
    if (rc != VBX_OK) return rc;
    if (block_capacity <= m->capacity) {
        if (s.error == VBX_ERR_POOL_FULL) return vbx_map_clear_error(m);
        return VBX_OK;
    }
    // copy the old hash to the host, allocate the bigger storage, move the pool, rehash
    std::vector<u64> okeys(m->hcap);
    std::vector<int> oslots(m->hcap);
    VBX_TRY(hipMemcpy(okeys.data(), m->hkeys, sizeof(u64) * m->hcap, hipMemcpyDeviceToHost));
    VBX_TRY(hipMemcpy(oslots.data(), m->hslots, sizeof(int) * m->hcap, hipMemcpyDeviceToHost));
    u64* old_keys = m->hkeys;
    int* old_slots = m->hslots;
    void* old_pool = m->pool;
    u32* old_color = m->color;
    const u32 old_cap = m->capacity;
    m->hkeys = nullptr;
    m->hslots = nullptr;
    m->pool = nullptr;
    m->color = nullptr;
    rc = alloc_storage(m, block_capacity);
    if (rc != VBX_OK) {
        free_storage(m);
        m->hkeys = old_keys;
        m->hslots = old_slots;
        m->pool = old_pool;
        m->color = old_color;
        m->capacity = old_cap;
        m->hcap = (u32)okeys.size();
        return rc;
    }
    VBX_TRY(hipMemcpyAsync(m->pool, old_pool, (size_t)s.block_count * 4096 * m->voxel_bytes,
                           hipMemcpyDeviceToDevice, m->stream));
    if (old_color)
        VBX_TRY(hipMemcpyAsync(m->color, old_color, (size_t)s.block_count * 4096 * sizeof(u32),
                               hipMemcpyDeviceToDevice, m->stream));
    std::vector<u64> nkeys(m->hcap, kEmpty);
    std::vector<int> nslots(m->hcap, 0);
    for (size_t i = 0; i < okeys.size(); ++i)
        if (okeys[i] != kEmpty) host_insert(nkeys, nslots, okeys[i], oslots[i]);
    VBX_TRY(hipStreamSynchronize(m->stream));
    VBX_TRY(hipMemcpy(m->hkeys, nkeys.data(), sizeof(u64) * m->hcap, hipMemcpyHostToDevice));
    VBX_TRY(hipMemcpy(m->hslots, nslots.data(), sizeof(int) * m->hcap, hipMemcpyHostToDevice));
    map_free(m, old_keys);
    map_free(m, old_slots);
    map_free(m, old_pool);
    map_free(m, old_color);
    m->P.block_capacity = block_capacity;
    if (m->esdf && (rc = esdf_grow_dirty(m)) != VBX_OK) return rc;
    if (s.error == VBX_ERR_POOL_FULL) {
        s.error = 0;
        VBX_TRY(hipMemcpy(m->st, &s, sizeof s, hipMemcpyHostToDevice));
    }
    return VBX_OK;
}

int vbx_export_blocks(vbx_map* m, int32_t* coords, float* dw, size_t cap, size_t* n_out) {
    if (!m || !n_out) return VBX_ERR_INVALID_ARG;
    MapState s;
    int rc = read_state(m, &s);
    if (rc != VBX_OK) return rc;
    const size_t nb = s.block_count;
    if (!coords && !dw) {
        *n_out = nb;
        return VBX_OK;
    }
    if (cap < nb) return VBX_ERR_BUFFER_TOO_SMALL;
    std::vector<u64> keys(m->hcap);
    std::vector<int> slots(m->hcap);
    VBX_TRY(hipMemcpy(keys.data(), m->hkeys, sizeof(u64) * m->hcap, hipMemcpyDeviceToHost));
    VBX_TRY(hipMemcpy(slots.data(), m->hslots, sizeof(int) * m->hcap, hipMemcpyDeviceToHost));
    std::vector<std::pair<u64, int>> blocks;
    blocks.reserve(nb);
    for (size_t i = 0; i < keys.size(); ++i)
        if (keys[i] != kEmpty) blocks.push_back({keys[i], slots[i]});
    if (blocks.size() != nb) return VBX_ERR_DEVICE;
    std::sort(blocks.begin(), blocks.end());
    std::vector<unsigned char> pool;
    if (dw) {
        pool.resize(nb * 4096 * m->voxel_bytes);
        if (nb) VBX_TRY(hipMemcpy(pool.data(), m->pool, pool.size(), hipMemcpyDeviceToHost));
    }
    for (size_t b = 0; b < nb; ++b) {
        if (coords) {
            int bx, by, bz;
            unpack_block(blocks[b].first, bx, by, bz);
            coords[3 * b] = bx;
            coords[3 * b + 1] = by;
            coords[3 * b + 2] = bz;
        }
        if (dw) {
            const size_t slot = (size_t)blocks[b].second;
            for (int l = 0; l < 4096; ++l) {
                float Dn, W;
                if (m->P.storage == VBX_F32) {
                    const float* v = (const float*)pool.data() + 2 * (slot * 4096 + l);
                    Dn = v[0];
                    W = v[1];
                } else {
                    const uint32_t raw = ((const uint32_t*)pool.data())[slot * 4096 + l];
                    const unsigned short dc = (unsigned short)(raw & 0xFFFF);
                    Dn = m->P.storage == VBX_F16 ? __half2float(__ushort_as_half(dc)) : s16_decode(dc);
                    W = __half2float(__ushort_as_half((unsigned short)(raw >> 16)));
                }
                dw[2 * (b * 4096 + l)] = m->P.storage == VBX_F32 ? Dn : Dn * m->P.trunc;
                dw[2 * (b * 4096 + l) + 1] = W;
            }
        }
    }
    *n_out = nb;
    return VBX_OK;
}

int vbx_export_colors(vbx_map* m, int32_t* coords, uint32_t* colors, size_t cap, size_t* n_out) {
    if (!m || !n_out) return VBX_ERR_INVALID_ARG;
    if (!m->color) return VBX_ERR_INVALID_ARG;
    MapState s;
    int rc = read_state(m, &s);
    if (rc != VBX_OK) return rc;
    const size_t nb = s.block_count;
    if (!coords && !colors) {
        *n_out = nb;
        return VBX_OK;
    }
    if (cap < nb) return VBX_ERR_BUFFER_TOO_SMALL;
    std::vector<u64> keys(m->hcap);
    std::vector<int> slots(m->hcap);
    VBX_TRY(hipMemcpy(keys.data(), m->hkeys, sizeof(u64) * m->hcap, hipMemcpyDeviceToHost));
    VBX_TRY(hipMemcpy(slots.data(), m->hslots, sizeof(int) * m->hcap, hipMemcpyDeviceToHost));
    std::vector<std::pair<u64, int>> blocks;
    blocks.reserve(nb);
    for (size_t i = 0; i < keys.size(); ++i)
        if (keys[i] != kEmpty) blocks.push_back({keys[i], slots[i]});
    if (blocks.size() != nb) return VBX_ERR_DEVICE;
    std::sort(blocks.begin(), blocks.end());
    std::vector<u32> pool;
    if (colors) {
        pool.resize(nb * 4096);
        if (nb) VBX_TRY(hipMemcpy(pool.data(), m->color, pool.size() * sizeof(u32), hipMemcpyDeviceToHost));
    }
    for (size_t b = 0; b < nb; ++b) {
        if (coords) {
            int bx, by, bz;
            unpack_block(blocks[b].first, bx, by, bz);
            coords[3 * b] = bx;
            coords[3 * b + 1] = by;
            coords[3 * b + 2] = bz;
        }
        if (colors)
            std::memcpy(colors + b * 4096, pool.data() + (size_t)blocks[b].second * 4096, 4096 * sizeof(u32));
    }
    *n_out = nb;
    return VBX_OK;
}

int vbx_import_blocks(vbx_map* m, const int32_t* coords, const float* dw, size_t n) {
    if (!m || (n > 0 && (!coords || !dw))) return VBX_ERR_INVALID_ARG;
    if (n > m->capacity) return VBX_ERR_POOL_FULL;
    MapState s;
    int rc = read_state(m, &s);
    if (rc != VBX_OK) return rc;
    std::vector<u64> keys(m->hcap, kEmpty);
    std::vector<int> slots(m->hcap, 0);
    std::vector<unsigned char> pool(n * 4096 * m->voxel_bytes);
    for (size_t b = 0; b < n; ++b) {
        const int bx = coords[3 * b], by = coords[3 * b + 1], bz = coords[3 * b + 2];
        const int lim = kVoxLimit / 16;
        if (bx < -lim || bx >= lim || by < -lim || by >= lim || bz < -lim || bz >= lim) return VBX_ERR_INVALID_ARG;
        host_insert(keys, slots, pack_block(bx, by, bz), (int)b);
        encode_block(m, dw + 2 * b * 4096, pool.data() + b * 4096 * m->voxel_bytes);
    }
    VBX_TRY(hipMemcpy(m->hkeys, keys.data(), sizeof(u64) * m->hcap, hipMemcpyHostToDevice));
    VBX_TRY(hipMemcpy(m->hslots, slots.data(), sizeof(int) * m->hcap, hipMemcpyHostToDevice));
    if (n) VBX_TRY(hipMemcpy(m->pool, pool.data(), pool.size(), hipMemcpyHostToDevice));
    s.block_count = (u32)n;
    s.new_count = 0;
    s.error = 0;
    VBX_TRY(hipMemcpy(m->st, &s, sizeof s, hipMemcpyHostToDevice));
    esdf_reset(m, n);      // new slots: the ESDF starts over from every imported block
    clear_colors(m);
    return VBX_OK;
}

int vbx_last_touches(vbx_map* m, int32_t* coords, uint32_t* counts, size_t cap, size_t* n_out) {
    if (!m || !n_out) return VBX_ERR_INVALID_ARG;
    if (!(m->P.flags & VBX_FLAG_KEEP_TOUCHES) || !m->touch_src) return VBX_ERR_INVALID_ARG;
    Scratch* s = m->touch_src;
    vbx_map* lead = s->last_maps.empty() ? m : s->last_maps[0];
    VBX_TRY(hipStreamSynchronize(lead->stream));
    CallState cs;
    VBX_TRY(hipMemcpy(&cs, s->cs.p, sizeof cs, hipMemcpyDeviceToHost));
    const size_t total = cs.touch_count;
    if (total > s->touch_cap) return VBX_ERR_BUFFER_TOO_SMALL;
    std::vector<u64> keys(total);
    std::vector<u32> n(total);
    if (total) {
        VBX_TRY(hipMemcpy(keys.data(), s->touch_key.p, total * sizeof(u64), hipMemcpyDeviceToHost));
        VBX_TRY(hipMemcpy(n.data(), s->touch_n.p, total * sizeof(u32), hipMemcpyDeviceToHost));
    }
    size_t cnt = 0;
    for (size_t i = 0; i < total; ++i)
        if ((int)(keys[i] >> 57) == m->touch_idx) ++cnt;
    if (!coords && !counts) {
        *n_out = cnt;
        return VBX_OK;
    }
    if (cap < cnt) return VBX_ERR_BUFFER_TOO_SMALL;
    size_t j = 0;
    for (size_t i = 0; i < total; ++i) {
        if ((int)(keys[i] >> 57) != m->touch_idx) continue;
        int gx, gy, gz;
        unpack_voxel(keys[i] & ((1ull << 57) - 1), gx, gy, gz);
        if (coords) {
            coords[3 * j] = gx;
            coords[3 * j + 1] = gy;
            coords[3 * j + 2] = gz;
        }
        if (counts) counts[j] = n[i];
        ++j;
    }
    *n_out = cnt;
    return VBX_OK;
}

int vbx_map_hash_stats(vbx_map* m, vbx_hash_stats* out) {
    if (!m || !out) return VBX_ERR_INVALID_ARG;
    VBX_TRY(hipStreamSynchronize(m->stream));
    std::vector<u64> keys(m->hcap);
    VBX_TRY(hipMemcpy(keys.data(), m->hkeys, sizeof(u64) * m->hcap, hipMemcpyDeviceToHost));
    const u32 mask = m->hcap - 1;
    uint64_t n = 0, sum = 0;
    uint32_t mx = 0;
    for (u32 i = 0; i < m->hcap; ++i) {
        if (keys[i] == kEmpty) continue;
        const u32 probe = ((i - ((u32)mix64(keys[i]) & mask)) & mask) + 1u;
        ++n;
        sum += probe;
        mx = probe > mx ? probe : mx;
    }
    out->slots = m->hcap;
    out->blocks = n;
    out->mean_probe = n ? (double)sum / (double)n : 0.0;
    out->max_probe = mx;
    out->reserved = 0;
    return VBX_OK;
}

int vbx_map_stats(vbx_map* m, vbx_stats* out) {
    if (!m || !out) return VBX_ERR_INVALID_ARG;
    MapState s;
    int rc = read_state(m, &s);
    if (rc != VBX_OK) return rc;
    out->points = s.points;
    out->valid = s.valid;
    out->invalid = s.invalid;
    out->out_of_bounds = s.oob;
    out->rays = s.rays;
    out->touches = s.touches;
    out->voxels = s.voxels;
    out->cells = s.cells;
    out->new_blocks = s.new_blocks;
    out->blocks = s.block_count;
    out->calls = s.calls;
    return VBX_OK;
}

int vbx_map_interpolate(vbx_map* m, const float* points_dev, size_t n, float* dist_dev) {
    if (!m || (n > 0 && (!points_dev || !dist_dev))) return VBX_ERR_INVALID_ARG;
    if (n > (size_t)VBX_MAX_QUERY_POINTS) return VBX_ERR_LIMIT;
    if (n == 0) return VBX_OK;
    const MapDesc d = make_desc(m, 0, 0, 0);
    const unsigned grid = grid_for(n, 8192);
    if (m->P.storage == VBX_F32)
        hipLaunchKernelGGL(k_interpolate<0>, dim3(grid), dim3(256), 0, m->stream, d, points_dev, (u32)n, dist_dev);
    else if (m->P.storage == VBX_F16)
        hipLaunchKernelGGL(k_interpolate<1>, dim3(grid), dim3(256), 0, m->stream, d, points_dev, (u32)n, dist_dev);
    else
        hipLaunchKernelGGL(k_interpolate<2>, dim3(grid), dim3(256), 0, m->stream, d, points_dev, (u32)n, dist_dev);
    return hipGetLastError() == hipSuccess ? VBX_OK : VBX_ERR_DEVICE;
}

int vbx_debug_traverse(const float* A_dev, const float* B_dev, int n, int32_t* out_dev, int cap,
                       int32_t* counts_dev) {
    if (n < 0 || cap < 0 || (n > 0 && (!A_dev || !B_dev || !counts_dev || (cap > 0 && !out_dev))))
        return VBX_ERR_INVALID_ARG;
    if (n == 0) return VBX_OK;
    hipLaunchKernelGGL(k_debug_traverse, dim3((n + 255) / 256), dim3(256), 0, nullptr, A_dev, B_dev, n,
                       (int*)out_dev, cap, (int*)counts_dev);
    VBX_TRY(hipGetLastError());
    VBX_TRY(hipStreamSynchronize(nullptr));
    return VBX_OK;
}

int vbx_debug_traverse_blocks(const float* A_dev, const float* B_dev, int n, int32_t* out_dev, int cap,
                              int32_t* counts_dev) {
    if (n < 0 || cap < 0 || (n > 0 && (!A_dev || !B_dev || !counts_dev || (cap > 0 && !out_dev))))
        return VBX_ERR_INVALID_ARG;
    if (n == 0) return VBX_OK;
    hipLaunchKernelGGL(k_debug_traverse_blocks, dim3((n + 255) / 256), dim3(256), 0, nullptr, A_dev, B_dev, n,
                       (int*)out_dev, cap, (int*)counts_dev);
    VBX_TRY(hipGetLastError());
    VBX_TRY(hipStreamSynchronize(nullptr));
    return VBX_OK;
}

int vbx_map_clear(vbx_map* m) {
    if (!m) return VBX_ERR_INVALID_ARG;
    hipLaunchKernelGGL(k_map_clear, dim3(grid_for(m->hcap)), dim3(256), 0, m->stream, m->hkeys, (size_t)m->hcap,
                       (u32*)m->st, (u32)(sizeof(MapState) / 4));
    esdf_reset(m, 0);
    clear_colors(m);
    VBX_TRY(hipGetLastError());
    return VBX_OK;
}

int vbx_write_blocks(vbx_map* m, const int32_t* coords, const float* dw, size_t n) {
    if (!m || (n > 0 && (!coords || !dw))) return VBX_ERR_INVALID_ARG;
    if (n == 0) return VBX_OK;
    MapState s;
    int rc = read_state(m, &s);
    if (rc != VBX_OK) return rc;
    std::vector<u64> keys(m->hcap);
    std::vector<int> slots(m->hcap);
    VBX_TRY(hipMemcpy(keys.data(), m->hkeys, sizeof(u64) * m->hcap, hipMemcpyDeviceToHost));
    VBX_TRY(hipMemcpy(slots.data(), m->hslots, sizeof(int) * m->hcap, hipMemcpyDeviceToHost));
    // the slot of every block: the one it holds, or the next free one
    std::vector<int> where(n);
    u32 count = s.block_count;
    const int lim = kVoxLimit / 16;
    for (size_t b = 0; b < n; ++b) {
        const int bx = coords[3 * b], by = coords[3 * b + 1], bz = coords[3 * b + 2];
        if (bx < -lim || bx >= lim || by < -lim || by >= lim || bz < -lim || bz >= lim) return VBX_ERR_INVALID_ARG;
        const u64 key = pack_block(bx, by, bz);
        const u32 mask = m->hcap - 1;
        u32 h = (u32)mix64(key) & mask;
        while (keys[h] != kEmpty && keys[h] != key) h = (h + 1) & mask;
        if (keys[h] == key) {
            where[b] = slots[h];
        } else {
            if (count >= m->capacity) return VBX_ERR_POOL_FULL;    // nothing written yet
            keys[h] = key;
            slots[h] = (int)count;
            where[b] = (int)count++;
        }
    }
    std::vector<unsigned char> block(4096 * m->voxel_bytes);
    const u32 one = 1u;
    for (size_t b = 0; b < n; ++b) {
        encode_block(m, dw + 2 * b * 4096, block.data());
        VBX_TRY(hipMemcpy((char*)m->pool + (size_t)where[b] * 4096 * m->voxel_bytes, block.data(), block.size(),
                          hipMemcpyHostToDevice));
        if (m->esdf) VBX_TRY(hipMemcpy(m->esdf->dirty + where[b], &one, sizeof one, hipMemcpyHostToDevice));
    }
    VBX_TRY(hipMemcpy(m->hkeys, keys.data(), sizeof(u64) * m->hcap, hipMemcpyHostToDevice));
    VBX_TRY(hipMemcpy(m->hslots, slots.data(), sizeof(int) * m->hcap, hipMemcpyHostToDevice));
    s.block_count = count;
    VBX_TRY(hipMemcpy(m->st, &s, sizeof s, hipMemcpyHostToDevice));
    return VBX_OK;
}

int vbx_esdf_enable(vbx_map* m, const vbx_esdf_params* p) {
    if (!m || !p || m->esdf) return VBX_ERR_INVALID_ARG;
    if (!(p->gamma > 0.0f) || !std::isfinite(p->d_max) || !(p->d_max >= p->gamma)) return VBX_ERR_INVALID_ARG;
    MapState s;
    int rc = read_state(m, &s);
    if (rc != VBX_OK) return rc;
    m->esdf = new (std::nothrow) Esdf();
    if (!m->esdf) return VBX_ERR_OUT_OF_MEMORY;
    m->esdf->P = *p;
    if ((rc = esdf_grow_dirty(m)) != VBX_OK) {
        esdf_free(m);
        return rc;
    }
    // the blocks the map already holds are new to the layer
    if (s.block_count)
        hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(s.block_count)), dim3(256), 0, m->stream, m->esdf->dirty, 1u,
                           (size_t)s.block_count);
    VBX_TRY(hipStreamSynchronize(m->stream));
    return VBX_OK;
}

int vbx_esdf_update(vbx_map* m, vbx_esdf_stats* out) {
    if (!m || !m->esdf) return VBX_ERR_INVALID_ARG;
    Esdf* e = m->esdf;
    MapState s;
    int rc = read_state(m, &s);
    if (rc != VBX_OK) return rc;
    if (s.error) return s.error;
    const u32 nb = s.block_count;
    e->stats.dirty_blocks = 0;
    e->stats.raise_rounds = 0;
    e->stats.lower_rounds = 0;
    e->stats.updates++;
    e->stats.voxels = (uint64_t)nb * 4096;
    if (nb == 0) {
        if (out) *out = e->stats;
        return VBX_OK;
    }
    hipStream_t st = m->stream;
    if ((rc = esdf_grow_dirty(m)) != VBX_OK || (rc = esdf_grow_vox(m, nb)) != VBX_OK) return rc;
    const size_t nv = (size_t)nb * 4096;
    // stamps: grown buffers start at 0, which no tag takes; old tags are all below the next ones
    auto grow_zero = [&](DevBuf& b, size_t bytes) -> int {
        if (b.bytes >= bytes && b.p) return VBX_OK;
        if (dev_alloc(b, bytes) != VBX_OK) return VBX_ERR_OUT_OF_MEMORY;
        hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(bytes / 4)), dim3(256), 0, st, (u32*)b.p, 0u, bytes / 4);
        return VBX_OK;
    };
    if (grow_zero(e->rstamp, nv * 4) != VBX_OK || grow_zero(e->lstamp, nv * 4) != VBX_OK ||
        dev_alloc(e->list, (size_t)nb * 4) != VBX_OK || dev_alloc(e->nbr, (size_t)nb * 27 * 4) != VBX_OK ||
        dev_alloc(e->slot_key, (size_t)nb * 8) != VBX_OK || dev_alloc(e->raise0, nv * 4) != VBX_OK ||
        dev_alloc(e->raise1, nv * 4) != VBX_OK || dev_alloc(e->lower0, nv * 4) != VBX_OK ||
        dev_alloc(e->lower1, nv * 4) != VBX_OK || dev_alloc(e->cnt, kEsdfCounters * 4) != VBX_OK)
        return VBX_ERR_OUT_OF_MEMORY;
    EsdfDev E;
    E.vox = e->vox;
    E.rstamp = (u32*)e->rstamp.p;
    E.lstamp = (u32*)e->lstamp.p;
    E.list = (u32*)e->list.p;
    E.nbr = (int*)e->nbr.p;
    E.raise[0] = (u32*)e->raise0.p;
    E.raise[1] = (u32*)e->raise1.p;
    E.lower[0] = (u32*)e->lower0.p;
    E.lower[1] = (u32*)e->lower1.p;
    E.cnt = (u32*)e->cnt.p;
    E.fcap = (u32)nv;
    E.gamma = e->P.gamma;
    E.d_max = e->P.d_max;
    const float v = m->P.voxel_size;
    E.step[0] = 0.0f;
    E.step[1] = v;
    E.step[2] = (float)((double)v * std::sqrt(2.0));
    E.step[3] = (float)((double)v * std::sqrt(3.0));
    const MapDesc d = make_desc(m, 0, 0, 0);
    // neighbour blocks of every block, rebuilt when blocks were added (new blocks change their
    // neighbours' tables too); blocks only come and go together with a reset otherwise
    if (e->nbr_blocks != nb) {
        hipLaunchKernelGGL(k_esdf_slot_keys, dim3(grid_for(m->hcap)), dim3(256), 0, st, m->hkeys, m->hslots,
                           m->hcap, (u64*)e->slot_key.p);
        hipLaunchKernelGGL(k_esdf_neighbours, dim3(grid_for((size_t)nb * 27)), dim3(256), 0, st, d,
                           (const u64*)e->slot_key.p, nb, (int*)e->nbr.p);
        e->nbr_blocks = nb;
    }
    hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(256), 0, st, E.cnt, 0u, (size_t)kEsdfCounters);
    hipLaunchKernelGGL(k_esdf_dirty_list, dim3(grid_for(nb)), dim3(256), 0, st, e->dirty, nb, E.list,
                       E.cnt + kEsdfDirtyCount);
    const unsigned G = 2048;   // persistent grids: threads stride over the frontier
    const u32 tag_raise0 = ++e->tag, tag_lower0 = ++e->tag;
    if (m->P.storage == VBX_F32)
        hipLaunchKernelGGL(k_esdf_seed<0>, dim3(G), dim3(256), 0, st, d, E, tag_raise0, tag_lower0);
    else if (m->P.storage == VBX_F16)
        hipLaunchKernelGGL(k_esdf_seed<1>, dim3(G), dim3(256), 0, st, d, E, tag_raise0, tag_lower0);
    else
        hipLaunchKernelGGL(k_esdf_seed<2>, dim3(G), dim3(256), 0, st, d, E, tag_raise0, tag_lower0);
    VBX_TRY(hipGetLastError());
    // levels in chunks, the host reading the frontier sizes between chunks; a level whose
    // frontier is empty returns at once
    constexpr u32 kChunk = 8;
    u32 host_cnt[kEsdfCounters];
    VBX_TRY(hipMemcpyAsync(host_cnt, E.cnt, sizeof host_cnt, hipMemcpyDeviceToHost, st));
    VBX_TRY(hipStreamSynchronize(st));
    u32 r = 0;
    while (host_cnt[kEsdfRaiseCount + r % 3] != 0) {
        for (u32 k = 0; k < kChunk; ++k, ++r)
            hipLaunchKernelGGL(k_esdf_raise, dim3(G), dim3(256), 0, st, E, r, ++e->tag, tag_lower0);
        VBX_TRY(hipMemcpyAsync(host_cnt, E.cnt, sizeof host_cnt, hipMemcpyDeviceToHost, st));
        VBX_TRY(hipStreamSynchronize(st));
    }
    e->stats.dirty_blocks = host_cnt[kEsdfDirtyCount];
    e->stats.raise_rounds = r;
    r = 0;
    while (host_cnt[kEsdfLowerCount + r % 3] != 0) {
        for (u32 k = 0; k < kChunk; ++k, ++r)
            hipLaunchKernelGGL(k_esdf_lower, dim3(G), dim3(256), 0, st, E, r, ++e->tag);
        VBX_TRY(hipMemcpyAsync(host_cnt, E.cnt, sizeof host_cnt, hipMemcpyDeviceToHost, st));
        VBX_TRY(hipStreamSynchronize(st));
    }
    e->stats.lower_rounds = r;
    VBX_TRY(hipGetLastError());
    if (out) *out = e->stats;
    return VBX_OK;
}

int vbx_esdf_export(vbx_map* m, int32_t* coords, float* d, uint8_t* info, size_t cap, size_t* n_out) {
    if (!m || !n_out || !m->esdf) return VBX_ERR_INVALID_ARG;
    MapState s;
    int rc = read_state(m, &s);
    if (rc != VBX_OK) return rc;
    const size_t nb = s.block_count;
    if ((coords || d || info) && cap < nb) return VBX_ERR_BUFFER_TOO_SMALL;
    if (!coords && !d && !info) {
        *n_out = nb;
        return VBX_OK;
    }
    std::vector<u64> keys(m->hcap);
    std::vector<int> slots(m->hcap);
    VBX_TRY(hipMemcpy(keys.data(), m->hkeys, sizeof(u64) * m->hcap, hipMemcpyDeviceToHost));
    VBX_TRY(hipMemcpy(slots.data(), m->hslots, sizeof(int) * m->hcap, hipMemcpyDeviceToHost));
    std::vector<std::pair<u64, int>> blocks;
    for (size_t i = 0; i < keys.size(); ++i)
        if (keys[i] != kEmpty) blocks.push_back({keys[i], slots[i]});
    if (blocks.size() != nb) return VBX_ERR_DEVICE;
    std::sort(blocks.begin(), blocks.end());
    std::vector<u64> words;
    const size_t have = std::min(m->esdf->vox_blocks, nb);
    words.assign(nb * 4096, 0ull);
    if (have) VBX_TRY(hipMemcpy(words.data(), m->esdf->vox, have * 4096 * sizeof(u64), hipMemcpyDeviceToHost));
    for (size_t b = 0; b < nb; ++b) {
        if (coords) {
            int bx, by, bz;
            unpack_block(blocks[b].first, bx, by, bz);
            coords[3 * b] = bx;
            coords[3 * b + 1] = by;
            coords[3 * b + 2] = bz;
        }
        const size_t slot = (size_t)blocks[b].second;
        for (int l = 0; l < 4096; ++l) {
            const u64 w = words[slot * 4096 + l];
            const u32 low = (u32)w;
            float mag;
            const u32 hi = (u32)(w >> 32);
            std::memcpy(&mag, &hi, 4);
            const bool obs = (low & kEsdfObserved) != 0;
            if (d) d[b * 4096 + l] = obs ? ((low & kEsdfNeg) ? -mag : mag) : 0.0f;
            if (info)
                info[b * 4096 + l] = obs ? (uint8_t)(1u | ((low & kEsdfFixed) ? 2u : 0u) |
                                                     ((low & kEsdfParentMask) << 2) | ((low & kEsdfNeg) ? 128u : 0u))
                                         : (uint8_t)0;
        }
    }
    *n_out = nb;
    return VBX_OK;
}

int vbx_map_profile(vbx_map* m, int enable) {
    if (!m) return VBX_ERR_INVALID_ARG;
    m->prof.mask = enable != 0 ? (1u << VBX_PROFILE_STAGES) - 1u : 0u;
    return VBX_OK;
}

int vbx_map_profile_stages(vbx_map* m, uint32_t stage_mask) {
    if (!m || (stage_mask >> VBX_PROFILE_STAGES) != 0) return VBX_ERR_INVALID_ARG;
    m->prof.mask = stage_mask;
    return VBX_OK;
}

int vbx_map_profile_read(vbx_map* m, vbx_profile* out, int reset) {
    if (!m || !out) return VBX_ERR_INVALID_ARG;
    VBX_TRY(hipStreamSynchronize(m->stream));
    for (const Profiler::Rec& r : m->prof.pending) {
        float ms = 0.0f;
        VBX_TRY(hipEventElapsedTime(&ms, r.a, r.b));
        m->prof.ms[r.stage] += ms;
        m->prof.launches[r.stage] += 1;
        m->prof.spare.push_back(r.a);
        m->prof.spare.push_back(r.b);
    }
    m->prof.pending.clear();
    for (int i = 0; i < VBX_PROFILE_STAGES; ++i) {
        out->ms[i] = m->prof.ms[i];
        out->launches[i] = m->prof.launches[i];
        if (reset) {
            m->prof.ms[i] = 0.0;
            m->prof.launches[i] = 0;
        }
    }
    return VBX_OK;
}

const char* vbx_profile_stage_name(int stage) {
    static const char* names[VBX_PROFILE_STAGES] = {"points", "groups", "cross", "resolve", "commit",
                                                    "bins", "scan", "scatter", "update", "finish"};
    return stage >= 0 && stage < VBX_PROFILE_STAGES ? names[stage] : nullptr;
}

int vbx_map_get_tuning(vbx_map* m, vbx_tuning* out) {
    if (!m || !out) return VBX_ERR_INVALID_ARG;
    std::memset(out, 0, sizeof *out);
    out->update_split = kUpdateVariants[m->update_variant].split;
    out->update_threads = kUpdateVariants[m->update_variant].threads;
    out->update_columns = kUpdateVariants[m->update_variant].columns;
    return VBX_OK;
}

int vbx_map_set_tuning(vbx_map* m, const vbx_tuning* t) {
    if (!m || !t) return VBX_ERR_INVALID_ARG;
    for (int v = 0; v < kNumUpdateVariants; ++v) {
        if (kUpdateVariants[v].split == t->update_split && kUpdateVariants[v].threads == t->update_threads &&
            kUpdateVariants[v].columns == (t->update_columns != 0)) {
            m->update_variant = v;
            return VBX_OK;
        }
    }
    return VBX_ERR_INVALID_ARG;
}

int vbx_map_autotune(vbx_map* m, const vbx_frame* frames, int F, vbx_tuning* best, double* ms_out) {
    if (!m || F <= 0 || !frames) return VBX_ERR_INVALID_ARG;
    vbx_map_params p = m->P;
    p.flags &= ~(uint32_t)VBX_FLAG_KEEP_TOUCHES;
    vbx_map* tmp = nullptr;
    int rc = vbx_map_create_ex(&p, &tmp);
    if (rc != VBX_OK) return rc;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        vbx_map_destroy(tmp);
        return VBX_ERR_DEVICE;
    }
    double best_ms = 1e300;
    int best_v = m->update_variant;
    const int reps = 3;
    for (int c = 0; c < kNumUpdateVariants && rc == VBX_OK; ++c) {
        tmp->update_variant = c;
        // one untimed pass (scratch growth, first touch), then the timed passes
        if ((rc = vbx_map_clear(tmp)) != VBX_OK || (rc = vbx_integrate_frames(tmp, frames, F)) != VBX_OK) break;
        (void)hipEventRecord(e0, tmp->stream);
        for (int r = 0; r < reps && rc == VBX_OK; ++r) {
            if ((rc = vbx_map_clear(tmp)) == VBX_OK) rc = vbx_integrate_frames(tmp, frames, F);
        }
        (void)hipEventRecord(e1, tmp->stream);
        if (hipEventSynchronize(e1) != hipSuccess) { rc = VBX_ERR_DEVICE; break; }
        float ms = 0.0f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        const double per = (double)ms / reps;
        if (ms_out) ms_out[c] = per;
        MapState s;
        if (read_state(tmp, &s) != VBX_OK || s.error != 0) { rc = s.error ? s.error : VBX_ERR_DEVICE; break; }
        if (per < best_ms) { best_ms = per; best_v = c; }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    vbx_map_destroy(tmp);
    if (rc != VBX_OK) return rc;
    m->update_variant = best_v;
    if (best) vbx_map_get_tuning(m, best);
    return VBX_OK;
}

void vbx_graph_destroy(vbx_graph* g) {
    if (!g) return;
    if (!g->maps.empty()) (void)hipStreamSynchronize(g->maps[0]->stream);
    if (g->capture_stream) (void)hipStreamSynchronize(g->capture_stream);
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    if (g->capture_stream) (void)hipStreamDestroy(g->capture_stream);
    free_scratch(g->scratch);
    delete g;
}

int vbx_graph_create(vbx_map* const* maps, int M, const vbx_frame* frames, const int* owner, int F,
                     vbx_graph** out) {
    if (!maps || !frames || !out || M <= 0 || F <= 0) return VBX_ERR_INVALID_ARG;
    if (M > 127 || F > VBX_MAX_FRAMES_PER_CALL) return VBX_ERR_LIMIT;
    if (!owner && F != M) return VBX_ERR_INVALID_ARG;
    for (int i = 0; i < M; ++i) {
        if (!maps[i]) return VBX_ERR_INVALID_ARG;
        for (int j = 0; j < i; ++j)
            if (maps[j] == maps[i]) return VBX_ERR_INVALID_ARG;
    }
    vbx_graph* g = new (std::nothrow) vbx_graph();
    if (!g) return VBX_ERR_OUT_OF_MEMORY;
    g->maps.assign(maps, maps + M);
    g->frames.assign(frames, frames + F);
    g->owner.resize(F);
    for (int i = 0; i < F; ++i) {
        g->owner[i] = owner ? owner[i] : i;
        if (g->owner[i] < 0 || g->owner[i] >= M) {
            delete g;
            return VBX_ERR_INVALID_ARG;
        }
    }
    g->update_variant = maps[0]->update_variant;
    for (int m = 0; m < M; ++m) g->capacity.push_back(maps[m]->capacity);
    g->scratch = new (std::nothrow) Scratch();
    if (!g->scratch) {
        delete g;
        return VBX_ERR_OUT_OF_MEMORY;
    }
    Prepared pr;
    hipStream_t st = maps[0]->stream;
    int rc = prepare_call(g->maps, g->frames, g->owner, pr);
    if (rc == VBX_OK) rc = ensure_scratch(g->scratch, st, pr.plan, (int)pr.jobs.size(), M, pr.sum_capacity);
    g->sum_capacity = pr.sum_capacity;
    if (rc == VBX_OK && hipStreamSynchronize(st) != hipSuccess) rc = VBX_ERR_DEVICE;
    if (rc == VBX_OK && hipStreamCreateWithFlags(&g->capture_stream, hipStreamNonBlocking) != hipSuccess) {
        g->capture_stream = nullptr;
        rc = VBX_ERR_DEVICE;
    }
    if (rc == VBX_OK) {
        warm_launch_shapes();
        if (hipStreamBeginCapture(g->capture_stream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
            rc = VBX_ERR_DEVICE;
        } else {
            const int lrc = launch_call(g->scratch, g->capture_stream, pr.plan, (int)pr.jobs.size(), M,
                                        g->update_variant, nullptr);
            const hipError_t ec = hipStreamEndCapture(g->capture_stream, &g->graph);
            if (lrc != VBX_OK || ec != hipSuccess || !g->graph) rc = VBX_ERR_DEVICE;
        }
    }
    if (rc == VBX_OK && hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0) != hipSuccess) {
        g->exec = nullptr;
        rc = VBX_ERR_DEVICE;
    }
    if (rc != VBX_OK) {
        vbx_graph_destroy(g);
        return rc;
    }
    *out = g;
    return VBX_OK;
}

int vbx_graph_launch(vbx_graph* g, const vbx_frame* frames, int F) {
    if (!g) return VBX_ERR_INVALID_ARG;
    if (frames) {
        if (F != (int)g->frames.size()) return VBX_ERR_INVALID_ARG;
        for (int i = 0; i < F; ++i)
            if (frames[i].n != g->frames[i].n || frames[i].width != g->frames[i].width) return VBX_ERR_INVALID_ARG;
    }
    for (size_t m = 0; m < g->maps.size(); ++m)
        if (g->maps[m]->capacity != g->capacity[m]) return VBX_ERR_INVALID_ARG;   // storage moved
    std::vector<vbx_frame> next = g->frames;
    if (frames) next.assign(frames, frames + F);
    Prepared pr;
    int rc = prepare_call(g->maps, next, g->owner, pr);
    if (rc != VBX_OK) return rc;
    hipStream_t st = g->maps[0]->stream;
    if ((rc = stage_tables(g->scratch, st, pr)) != VBX_OK) return rc;
    VBX_TRY(hipGraphLaunch(g->exec, st));
    g->frames.swap(next);
    note_touches(g->scratch, g->maps, pr.plan);
    return VBX_OK;
}

double vbx_server_clock(void) { return server_clock(); }

int vbx_server_create(const vbx_server_params* params, vbx_server** out) {
    if (!params || !out || params->budget_bytes == 0) return VBX_ERR_INVALID_ARG;
    if (params->max_inflight < 0 || params->max_inflight >= kServerSlots) return VBX_ERR_INVALID_ARG;
    vbx_server* S = new (std::nothrow) vbx_server();
    if (!S) return VBX_ERR_OUT_OF_MEMORY;
    S->P = *params;
    if (S->P.max_frames_per_tick == 0 || S->P.max_frames_per_tick > VBX_MAX_FRAMES_PER_CALL)
        S->P.max_frames_per_tick = 256;
    if (S->P.max_points_per_tick == 0) S->P.max_points_per_tick = (uint64_t)1 << 24;
    if (S->P.max_inflight == 0) S->P.max_inflight = 2;
    S->planner = vbx_sched::Planner(params->budget_bytes);
    (void)hipGetDevice(&S->device);
    int rc = VBX_OK;
    if (params->stream) {
        S->stream = (hipStream_t)params->stream;
    } else if (hipStreamCreate(&S->stream) == hipSuccess) {   // orders after null-stream uploads
        S->own_stream = true;
    } else {
        rc = VBX_ERR_DEVICE;
    }
    S->scratch = new (std::nothrow) Scratch();
    if (rc == VBX_OK && !S->scratch) rc = VBX_ERR_OUT_OF_MEMORY;
    if (rc == VBX_OK && hipMalloc(&S->status_dev, sizeof(int) * 128 * kServerSlots) != hipSuccess) {
        S->status_dev = nullptr;
        rc = VBX_ERR_OUT_OF_MEMORY;
    }
    if (rc == VBX_OK && hipHostMalloc(&S->status_host, sizeof(int) * 128 * kServerSlots, hipHostMallocDefault) !=
                            hipSuccess) {
        S->status_host = nullptr;
        rc = VBX_ERR_OUT_OF_MEMORY;
    }
    if (rc != VBX_OK) {
        if (S->status_dev) (void)hipFree(S->status_dev);
        if (S->own_stream) (void)hipStreamDestroy(S->stream);
        free_scratch(S->scratch);
        delete S;
        return rc;
    }
    warm_launch_shapes();
    S->engine = std::thread(server_engine, S);
    S->completer = std::thread(server_completer, S);
    *out = S;
    return VBX_OK;
}

int vbx_server_add_map(vbx_server* S, const vbx_map_params* params, int* map_id) {
    if (!S || !params || !map_id) return VBX_ERR_INVALID_ARG;
    int rc = validate_params(*params);
    if (rc != VBX_OK) return rc;
    vbx_map_params p = *params;
    p.stream = S->stream;
    const uint64_t bytes = map_storage_bytes(p, p.block_capacity);
    int id = -1;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        if (!S->planner.admit(bytes, &id)) {
            S->rejected_maps++;
            return VBX_ERR_OUT_OF_MEMORY;
        }
        S->maps.push_back(nullptr);
    }
    vbx_map* m = nullptr;
    rc = vbx_map_create_ex(&p, &m);
    std::lock_guard<std::mutex> lk(S->mu);
    if (rc != VBX_OK) {
        // the budget stays charged to a slot that never receives requests
        S->rejected_maps++;
        return rc;
    }
    S->maps[(size_t)id] = m;
    *map_id = id;
    return VBX_OK;
}

int vbx_server_submit(vbx_server* S, int map_id, const vbx_frame* frame, double t_arrival, uint64_t* ticket) {
    if (!S || !frame) return VBX_ERR_INVALID_ARG;
    if (frame->n > VBX_MAX_POINTS_PER_FRAME) return VBX_ERR_LIMIT;
    if ((frame->n > 0 && !frame->points) || (frame->width > 0 && frame->n % frame->width != 0))
        return VBX_ERR_INVALID_ARG;
    for (int q = 0; q < 12; ++q)
        if (!std::isfinite(frame->pose[q])) return VBX_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(S->mu);
    if (map_id < 0 || map_id >= (int)S->maps.size() || !S->maps[(size_t)map_id]) return VBX_ERR_INVALID_ARG;
    S->entries.emplace_back();
    ServerEntry& e = S->entries.back();
    e.frame = *frame;
    e.req.ticket = S->entries.size();
    e.req.map = map_id;
    e.req.points = frame->n;
    e.req.t_arrival = t_arrival > 0.0 ? t_arrival : server_clock();
    S->planner.submit(&e.req);
    S->submitted++;
    if (ticket) *ticket = e.req.ticket;
    S->cv_engine.notify_one();
    return VBX_OK;
}

int vbx_server_wait(vbx_server* S, uint64_t ticket, int* status, double* t_done) {
    if (!S) return VBX_ERR_INVALID_ARG;
    std::unique_lock<std::mutex> lk(S->mu);
    if (ticket == 0 || ticket > S->entries.size()) return VBX_ERR_INVALID_ARG;
    vbx_sched::Request& r = S->entries[(size_t)(ticket - 1)].req;
    S->cv_done.wait(lk, [&] { return r.state == 2; });
    if (status) *status = r.status;
    if (t_done) *t_done = r.t_done;
    return VBX_OK;
}

int vbx_server_drain(vbx_server* S) {
    if (!S) return VBX_ERR_INVALID_ARG;
    std::unique_lock<std::mutex> lk(S->mu);
    S->cv_done.wait(lk, [&] { return S->finished == S->submitted; });
    return VBX_OK;
}

int vbx_server_stats(vbx_server* S, vbx_server_summary* out) {
    if (!S || !out) return VBX_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(S->mu);
    std::memset(out, 0, sizeof *out);
    out->submitted = S->submitted;
    out->completed = S->finished - S->failed;
    out->failed = S->failed;
    out->ticks = S->ticks;
    out->frames = S->frames;
    out->points = S->points;
    out->replays = S->replays;
    out->maps = (uint32_t)S->planner.num_maps();
    out->rejected_maps = S->rejected_maps;
    out->budget_bytes = S->planner.budget();
    out->used_bytes = S->planner.used();
    out->mean_frames_per_tick = S->ticks ? (double)S->frames / (double)S->ticks : 0.0;
    std::vector<double> lat = S->latency;
    if (!lat.empty()) {
        std::sort(lat.begin(), lat.end());
        auto pct = [&](double q) {
            const size_t i = (size_t)std::min<double>((double)lat.size() - 1, std::ceil(q * (double)lat.size()) - 1);
            return lat[i] * 1e3;
        };
        out->p50_ms = pct(0.50);
        out->p99_ms = pct(0.99);
        out->max_ms = lat.back() * 1e3;
        double sum = 0.0;
        for (double x : lat) sum += x;
        out->mean_ms = sum / (double)lat.size() * 1e3;
        if (S->last_done > S->first_arrival)
            out->points_per_s = (double)S->points / (S->last_done - S->first_arrival);
    }
    return VBX_OK;
}

int vbx_server_reset_stats(vbx_server* S) {
    if (!S) return VBX_ERR_INVALID_ARG;
    std::unique_lock<std::mutex> lk(S->mu);
    S->cv_done.wait(lk, [&] { return S->finished == S->submitted; });
    S->submitted = S->finished = S->failed = S->ticks = S->frames = S->points = S->replays = 0;
    S->first_arrival = 1e300;
    S->last_done = 0.0;
    S->latency.clear();
    return VBX_OK;
}

vbx_map* vbx_server_map(vbx_server* S, int map_id) {
    if (!S) return nullptr;
    std::lock_guard<std::mutex> lk(S->mu);
    if (map_id < 0 || map_id >= (int)S->maps.size()) return nullptr;
    return S->maps[(size_t)map_id];
}

void vbx_server_destroy(vbx_server* S) {
    if (!S) return;
    {
        std::unique_lock<std::mutex> lk(S->mu);
        S->cv_done.wait(lk, [&] { return S->finished == S->submitted; });
        S->stop = true;
    }
    S->cv_engine.notify_all();
    S->cv_complete.notify_all();
    if (S->engine.joinable()) S->engine.join();
    if (S->completer.joinable()) S->completer.join();
    (void)hipStreamSynchronize(S->stream);
    for (vbx_map* m : S->maps) vbx_map_destroy(m);
    for (hipEvent_t e : S->spare_events) (void)hipEventDestroy(e);
    for (TickRec& t : S->inflight)
        if (t.ev) (void)hipEventDestroy(t.ev);
    free_scratch(S->scratch);
    if (S->status_dev) (void)hipFree(S->status_dev);
    if (S->status_host) (void)hipHostFree(S->status_host);
    if (S->own_stream) (void)hipStreamDestroy(S->stream);
    delete S;
}

const char* vbx_status_string(int status) {
    switch (status) {
        case VBX_OK: return "ok";
        case VBX_ERR_INVALID_ARG: return "invalid argument";
        case VBX_ERR_OUT_OF_MEMORY: return "out of memory";
        case VBX_ERR_POOL_FULL: return "block pool full";
        case VBX_ERR_BUFFER_TOO_SMALL: return "buffer too small";
        case VBX_ERR_DEVICE: return "device error";
        case VBX_ERR_LIMIT: return "limit exceeded";
        default: return "unknown status";
    }
}

}  // extern "C"
