// Host-side internals shared by the kernels and the C-ABI implementation.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "vbx_internal.h"

namespace vbx {

// Per-frame counters of one call (device, zeroed after every call).
struct JobStat {
    u64 valid, invalid, oob_pts, oob_rays, rays, touches, voxels, cells;
};

// Kernels (defined in vbx_kernels.hip).
__global__ void k_fill_u64(u64* p, u64 val, size_t n);
__global__ void k_fill_u32(u32* p, u32 val, size_t n);
// Words of a host table passed by value in one launch's arguments.
constexpr int kTableChunkWords = 256;
struct TableChunk {
    u32 w[kTableChunkWords];
};
__global__ void k_set_u32(u32* p, u32 v);
__global__ void k_put_words(TableChunk c, u32 n, u32* dst);
__global__ void k_map_clear(u64* hkeys, size_t hcap, u32* state, u32 state_words);
__global__ void k_map_status(const MapDesc* maps, int nmaps, int* out);
// Colour calls pass the colour buffers (rays_c, parts_c, sorted_c, ...); other calls null.
__global__ void k_points_simple(const Job* jobs, int njobs, const MapDesc* maps, float4* rays_p,
                                u32* rays_job, u32* rays_c, JobStat* jst, CallState* cs);
template <bool COLOR>
__global__ void k_points_grouped(const Job* jobs, int njobs, const MapDesc* maps, u64* tkeys, u32 tmask,
                                 u32* tlist, u32 tlist_cap, Partial* parts, PartialColor* parts_c,
                                 u32* tile_parts, u32 tiles_per_job, JobStat* jst, CallState* cs);
__global__ void k_densify(const u32* tlist, u32 tlist_cap, u32* tval, const CallState* cs);
__global__ void k_gbin_count(const Partial* parts, const u32* tile_parts, u32 ntiles,
                             const u32* tval, u32* bins, u32 JM, u32 tpw, const CallState* cs);
__global__ void k_gscatter(const Partial* parts, const u32* tile_parts, u32 ntiles,
                           const u32* tval, u32* bins, const u32* off, u32 JM, u32 tpw,
                           Partial* sorted, const PartialColor* parts_c, PartialColor* sorted_c,
                           const CallState* cs);
template <bool COLOR>
__global__ void k_group_merge(const Job* jobs, const MapDesc* maps, const u64* tkeys,
                              const u32* tlist, const u32* off, const u32* chunk_first,
                              const Partial* sorted, u32 JM, const PartialColor* sorted_c, float4* rays_p,
                              u32* rays_job, u32* rays_c, JobStat* jst, CallState* cs);
__global__ void k_cross(const Job* jobs, const MapDesc* maps, const float4* rays_p,
                        const u32* rays_job, u64* tkeys, u32 tmask, u32* tlist, u32 tlist_cap,
                        u32* cross, unsigned char* ncross, u32 MB, u32* hbins, u32 JM, JobStat* jst,
                        CallState* cs, u32 ray_cap);
__global__ void k_resolve(const MapDesc* maps, const u64* tkeys, u32* tval, const u32* tlist,
                          u64* t_key, int* t_slot, CallState* cs);
__global__ void k_commit(const MapDesc* maps, const u64* t_key, int* t_slot, CallState* cs);
__global__ void k_bin_count(const Job* jobs, const u32* cross, const unsigned char* ncross,
                            u32 MB, const u32* tval, const u32* rays_job, u32* bins, u32 JM,
                            CallState* cs, u32 ray_cap);
__global__ void k_scan_sums(u32* bins, u32 JM, u32* partial, u32* off, CallState* cs, u32* hsrc,
                            const u32* tlist, u32 tlist_cap);
__global__ void k_scan_final(const u32* bins, const u32* partial, u32* off, u32 JM, u32* chunk_first,
                             const CallState* cs);
__global__ void k_scatter(const Job* jobs, const u32* cross, const unsigned char* ncross,
                          u32 MB, const u32* tval, const u32* rays_job, u32* bins,
                          const u32* off, u32 JM, const float4* rays_p, float4* sorted,
                          const u32* rays_c, u32* sorted_c, CallState* cs, u32 ray_cap);
template <int STORAGE, int RX, int RY, int RZ, int NT, bool COLOR>
__global__ void k_update(const Job* jobs, const MapDesc* maps, const u64* t_key, const int* t_slot,
                         const u32* off, const u32* order, const float4* sorted, const u32* sorted_c, u32 JM,
                         u64* touch_key, u32* touch_n, u32 touch_cap, int keep_touches, JobStat* jst,
                         CallState* cs);
__global__ void k_order_blocks(const u32* off, u32 JM, u32* order, const CallState* cs);
__global__ void k_finish_call(const Job* jobs, const MapDesc* maps, int nmaps, JobStat* jst, u64* tkeys,
                              u32 tkey_cap, const u32* tlist, u32 tlist_cap, CallState* cs);
template <int STORAGE>
__global__ void k_interpolate(const MapDesc M, const float* q, u32 n, float* out);

// Pinhole intrinsics of projection mapping: pixel coordinates u = fx x / z + cx, v = fy y / z + cy.
struct Intrinsics {
    float fx, fy, cx, cy;
};
template <int STORAGE>
__global__ void k_project(const Job* jobs, const MapDesc* maps, const u64* t_key, const int* t_slot, u32* bins,
                          u32 JM, Intrinsics K,
                          u64* touch_key, u32* touch_n, u32 touch_cap, int keep_touches, JobStat* jst,
                          CallState* cs);
__global__ void k_debug_traverse(const float* A, const float* B, int n, int* out, int cap,
                                 int* counts);
__global__ void k_debug_traverse_blocks(const float* A, const float* B, int n, int* out, int cap,
                                 int* counts);

constexpr int kScanChunkHost = 4096;

// ESDF layer (Sec. V-A): one 64-bit word per voxel, |d| in the high half, flags and parent below.
constexpr u32 kEsdfNeg = 1u << 31, kEsdfObserved = 1u << 30, kEsdfFixed = 1u << 29;
constexpr u32 kEsdfParentMask = 31u, kEsdfNoParent = 13u;
enum { kEsdfRaiseCount = 0, kEsdfLowerCount = 3, kEsdfDirtyCount = 6, kEsdfCounters = 8 };

// Device view of a map's ESDF layer for one update.
struct EsdfDev {
    u64* vox;        // [blocks * 4096] voxel words
    u32* rstamp;     // [blocks * 4096] last raise-frontier tag per voxel
    u32* lstamp;     // [blocks * 4096] last lower-frontier tag per voxel
    u32* list;       // [blocks] dirty blocks of this update
    int* nbr;        // [blocks * 27] neighbour block slots (-1: none)
    u32* raise[2];   // raise frontiers (voxel ids slot << 12 | local)
    u32* lower[2];   // lower frontiers
    u32* cnt;        // [kEsdfCounters]
    u32 fcap;        // frontier capacity (voxels)
    float gamma, d_max;
    float step[4];   // step length by squared offset length: 0, v, sqrt(2) v, sqrt(3) v
};

__global__ void k_esdf_slot_keys(const u64* hkeys, const int* hslots, u32 hcap, u64* slot_key);
__global__ void k_esdf_neighbours(const MapDesc M, const u64* slot_key, u32 nblocks, int* nbr);
__global__ void k_esdf_dirty_list(u32* dirty, u32 nblocks, u32* list, u32* count);
template <int STORAGE>
__global__ void k_esdf_seed(const MapDesc M, EsdfDev E, u32 tag_raise, u32 tag_lower);
__global__ void k_esdf_raise(EsdfDev E, u32 r, u32 tag_next, u32 tag_lower);
__global__ void k_esdf_lower(EsdfDev E, u32 r, u32 tag_next);

}  // namespace vbx
