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
__global__ void k_points_simple(const Job* jobs, int njobs, const MapDesc* maps, float4* rays_p,
                                u32* rays_job, JobStat* jst, CallState* cs);
__global__ void k_points_grouped(const Job* jobs, int njobs, const MapDesc* maps, u64* tkeys, u32 tmask,
                                 u32* tlist, u32 tlist_cap, Partial* parts, u32* tile_parts, u32 tiles_per_job,
                                 JobStat* jst, CallState* cs);
__global__ void k_densify(const u32* tlist, u32 tlist_cap, u32* tval, const CallState* cs);
__global__ void k_gbin_count(const Partial* parts, const u32* tile_parts, u32 ntiles,
                             const u32* tval, u32* bins, u32 JM, u32 tpw, const CallState* cs);
__global__ void k_gscatter(const Partial* parts, const u32* tile_parts, u32 ntiles,
                           const u32* tval, u32* bins, const u32* off, u32 JM, u32 tpw,
                           Partial* sorted, const CallState* cs);
__global__ void k_group_merge(const Job* jobs, const MapDesc* maps, const u64* tkeys,
                              const u32* tlist, const u32* off, const u32* chunk_first,
                              const Partial* sorted, u32 JM, float4* rays_p, u32* rays_job,
                              JobStat* jst, CallState* cs);
__global__ void k_cross(const Job* jobs, const MapDesc* maps, const float4* rays_p,
                        const u32* rays_job, u64* tkeys, u32 tmask, u32* tlist, u32 tlist_cap,
                        u32* cross, unsigned char* ncross, u32 MB, JobStat* jst, CallState* cs,
                        u32 ray_cap);
__global__ void k_resolve(const MapDesc* maps, const u64* tkeys, u32* tval, const u32* tlist,
                          u64* t_key, int* t_slot, CallState* cs);
__global__ void k_commit(const MapDesc* maps, const u64* t_key, int* t_slot, CallState* cs);
__global__ void k_bin_count(const Job* jobs, const u32* cross, const unsigned char* ncross,
                            u32 MB, const u32* tval, const u32* rays_job, u32* bins, u32 JM,
                            CallState* cs, u32 ray_cap);
__global__ void k_scan_sums(const u32* bins, u32 JM, u32* partial, u32* off, CallState* cs);
__global__ void k_scan_final(const u32* bins, const u32* partial, u32* off, u32 JM, u32* chunk_first,
                             const CallState* cs);
__global__ void k_scatter(const Job* jobs, const u32* cross, const unsigned char* ncross,
                          u32 MB, const u32* tval, const u32* rays_job, u32* bins,
                          const u32* off, u32 JM, const float4* rays_p, float4* sorted,
                          CallState* cs, u32 ray_cap);
template <int STORAGE, int RX, int RY, int RZ, int NT>
__global__ void k_update(const Job* jobs, const MapDesc* maps, const u64* t_key, const int* t_slot,
                         const u32* off, const u32* order, const float4* sorted, u32 JM, u64* touch_key,
                         u32* touch_n, u32 touch_cap, int keep_touches, JobStat* jst, CallState* cs);
__global__ void k_order_blocks(const u32* off, u32 JM, u32* order, const CallState* cs);
__global__ void k_finish_call(const Job* jobs, const MapDesc* maps, int nmaps, JobStat* jst, u64* tkeys,
                              u32 tkey_cap, const u32* tlist, u32 tlist_cap, CallState* cs);
template <int STORAGE>
__global__ void k_interpolate(const MapDesc M, const float* q, u32 n, float* out);
__global__ void k_debug_traverse(const float* A, const float* B, int n, int* out, int cap,
                                 int* counts);

constexpr int kScanChunkHost = 4096;

}  // namespace vbx
