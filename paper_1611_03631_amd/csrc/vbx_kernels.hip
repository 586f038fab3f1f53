// HIP kernels of the vbx TSDF integrator (gfx950, wave64).
//
// One integration call runs this pipeline on the map's stream:
//   points   : validity, pose transform, voxel keying (one thread per point, coalesced
//              12-byte loads).  Per-point raycasting writes one ray per valid point.
//              Grouped raycasting (Sec. IV-B) merges the points of a tile in an LDS hash by
//              voxel and writes one record per partial group, tagged with its block.
//   groups   : (grouped only) counting sort of the partial groups by (block, frame), then
//              one workgroup per bin merges them by voxel in LDS and casts one ray per
//              group; every sum is an exact integer, so the order never matters.
//   cross    : walk every ray through its truncation band and record, for each block the
//              walk enters, a (block, ray) crossing; blocks are collected in a per-call hash.
//   resolve  : look the call's blocks up in the map's block hash (wavefront-cooperative
//              probing), count the blocks that are new.
//   commit   : if the pool has room for all new blocks, insert them (all or nothing).
//   bins     : counting sort of the crossings by (block, frame): count, scan, scatter.
//   update   : one workgroup per touched block keeps the block's 4096 voxels in registers,
//              replays each frame's rays through the block into LDS accumulators (exact
//              fixed-point sums, so the result does not depend on the order of rays) and
//              applies Eqs. (3)-(4) once per voxel per frame, frame after frame.
//   finish   : commit block counts and statistics; clean the per-call tables.
#include "vbx_internal.h"
#include "vbx_host.h"

#include <hip/hip_fp16.h>

#pragma clang fp contract(off)

namespace vbx {

// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------
__device__ inline int lane_id() { return __lane_id(); }

// Adds the number of active lanes holding each distinct key to base[key]; one atomic per
// distinct key in the wave.  Must be reached by every lane still running in the wave.
__device__ inline void wave_count_by_key(u32* base, bool active, u32 key) {
    u64 pending = __ballot(active);
    const int lane = lane_id();
    while (pending) {
        int leader = __ffsll((long long)pending) - 1;
        u32 k = __shfl(key, leader);
        bool mine = ((pending >> lane) & 1ull) && key == k;
        u64 grp = __ballot(mine);
        if (lane == leader) atomicAdd(&base[k], (u32)__popcll(grp));
        pending &= ~grp;
    }
}

// Groups the active lanes of a wave by key (ballots only): each lane learns its group's first
// lane and its rank in the group, and that first lane the group's size.
__device__ inline void wave_group_by_key(bool active, u32 key, u32& leader_of, u32& rank, u32& count) {
    const int lane = lane_id();
    u64 pending = __ballot(active);
    leader_of = 0; rank = 0; count = 0;
    while (pending) {
        const int leader = __ffsll((long long)pending) - 1;
        const u32 kb = __shfl(key, leader);
        const bool mine = ((pending >> lane) & 1ull) && key == kb;
        const u64 grp = __ballot(mine);
        if (mine) {
            leader_of = (u32)leader;
            rank = (u32)__popcll(grp & ((1ull << lane) - 1ull));
        }
        if (lane == leader) count = (u32)__popcll(grp);
        pending &= ~grp;
    }
}

// Counting-sort positions for the active lanes of a wave: lanes with equal keys take
// consecutive positions below their bin's remaining count, reserved by one atomic per distinct
// key.  The groups are found first (ballots only) and every group's atomic is then issued by
// one instruction, so a wave waits for one atomic round trip rather than one per key.
__device__ inline u32 wave_claim_by_key(u32* bins, const u32* off, bool active, u32 key) {
    const u32 o = off[active ? key : 0u];   // loaded before the reservation, in flight with it
    u32 leader_of, rank, count;
    wave_group_by_key(active, key, leader_of, rank, count);
    u32 old = 0;
    if (count) old = atomicSub(&bins[key], count);   // the leaders, together
    const u32 base = (u32)__shfl((int)old, (int)leader_of);
    return active ? o + base - 1u - rank : 0u;
}

// The same for N keys per lane, all N sets of reservations in flight together.
template <int N>
__device__ inline void wave_claim_by_keys(u32* bins, const u32* off, const bool (&act)[N],
                                          const u32 (&key)[N], u32 (&pos)[N]) {
    u32 lead[N], rank[N], cnt[N], old[N], o[N];
#pragma unroll
    for (int k = 0; k < N; ++k) o[k] = off[act[k] ? key[k] : 0u];   // in flight with the reservations
#pragma unroll
    for (int k = 0; k < N; ++k) wave_group_by_key(act[k], key[k], lead[k], rank[k], cnt[k]);
#pragma unroll
    for (int k = 0; k < N; ++k) {
        old[k] = 0;
        if (cnt[k]) old[k] = atomicSub(&bins[key[k]], cnt[k]);
    }
#pragma unroll
    for (int k = 0; k < N; ++k) {
        const u32 base = (u32)__shfl((int)old[k], (int)lead[k]);
        pos[k] = act[k] ? o[k] + base - 1u - rank[k] : 0u;
    }
}

// Inclusive prefix sum over a 256-thread workgroup; returns the inclusive value, total in *tot.
__device__ inline u32 block_scan_256(u32 x, u32* lds8, u32* tot) {
    const int lane = lane_id(), wave = threadIdx.x >> 6;
    u32 v = x;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        u32 y = __shfl_up(v, o);
        if (lane >= o) v += y;
    }
    if (lane == 63) lds8[wave] = v;
    __syncthreads();
    u32 add = 0, total = 0;
#pragma unroll
    for (int w = 0; w < 4; ++w) {
        u32 s = lds8[w];
        if (w < wave) add += s;
        total += s;
    }
    __syncthreads();
    *tot = total;
    return v + add;
}

// Sum and OR over the 64 lanes of a wave (every lane active).
__device__ inline u32 wave_sum(u32 x) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += (u32)__shfl_xor((int)x, o);
    return x;
}
__device__ inline u64 wave_sum64(u64 x) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += (u64)__shfl_xor((long long)x, o);
    return x;
}
__device__ inline u32 wave_or(u32 x) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x |= (u32)__shfl_xor((int)x, o);
    return x;
}

// Inclusive count of the flagged threads of a 256-thread workgroup (ballots; lds4 holds four
// words); *tot = all flagged threads.
__device__ inline u32 block_count_256(bool flag, u32* lds4, u32* tot) {
    const int lane = lane_id(), wave = threadIdx.x >> 6;
    const u64 b = __ballot(flag);
    const u32 below = __builtin_amdgcn_mbcnt_hi((u32)(b >> 32), __builtin_amdgcn_mbcnt_lo((u32)b, 0u));
    if (lane == 0) lds4[wave] = (u32)__popcll(b);
    __syncthreads();
    u32 add = 0, total = 0;
#pragma unroll
    for (int w = 0; w < 4; ++w) {
        const u32 s = lds4[w];
        if (w < wave) add += s;
        total += s;
    }
    __syncthreads();
    *tot = total;
    return add + below + (flag ? 1u : 0u);
}

// Slot of a key in a small LDS table of 2^BITS slots: the top bits of a 32-bit multiplicative
// hash of the key's two halves.
template <int BITS>
__device__ inline u32 lds_slot(u64 key) {
    const u32 x = (u32)key ^ ((u32)(key >> 32) * 0x85EBCA6Bu);
    return (x * 0x9E3779B1u) >> (32 - BITS);
}

// Inclusive prefix sum over a workgroup of NT threads (NT a multiple of 64, at most 1024);
// lds needs NT / 64 entries.  Returns the inclusive value, the total in *tot.
template <int NT>
__device__ inline u32 block_scan(u32 x, u32* lds, u32* tot) {
    constexpr int NW = NT / 64;
    const int lane = lane_id(), wave = threadIdx.x >> 6;
    u32 v = x;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        u32 y = __shfl_up(v, o);
        if (lane >= o) v += y;
    }
    if (NW == 1) {
        *tot = __shfl(v, 63);
        return v;
    }
    if (lane == 63) lds[wave] = v;
    __syncthreads();
    u32 add = 0, total = 0;
#pragma unroll
    for (int w = 0; w < NW; ++w) {
        u32 s = lds[w];
        if (w < wave) add += s;
        total += s;
    }
    __syncthreads();
    *tot = total;
    return v + add;
}

__global__ void k_fill_u64(u64* p, u64 val, size_t n) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = val;
}
__global__ void k_fill_u32(u32* p, u32 val, size_t n) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = val;
}
__global__ void k_set_u32(u32* p, u32 v) { *p = v; }

// Writes n <= kTableChunkWords words carried in the kernel's arguments to dst: host tables reach
// the device in launch parameters, with no staging buffer.
__global__ void k_put_words(TableChunk c, u32 n, u32* dst) {
    for (u32 i = threadIdx.x; i < n; i += blockDim.x) dst[i] = c.w[i];
}
// Empties a map: every hash slot free, and (workgroup 0) its state words zero.
__global__ void k_map_clear(u64* hkeys, size_t hcap, u32* state, u32 state_words) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < hcap; i += (size_t)gridDim.x * blockDim.x)
        hkeys[i] = kEmpty;
    if (blockIdx.x == 0)
        for (u32 i = threadIdx.x; i < state_words; i += blockDim.x) state[i] = 0u;
}

// Status each map of a call was left in (maps of the staged table, in table order).
__global__ void k_map_status(const MapDesc* __restrict__ maps, int nmaps, int* __restrict__ out) {
    for (int m = threadIdx.x; m < nmaps; m += blockDim.x) out[m] = maps[m].st->error;
}

// Job of a tile: the last job whose first tile is <= tile (first tiles are non-decreasing),
// found with one round of loads and a vote.  Every lane of the wave must call it.
__device__ inline int job_of_tile(const Job* jobs, int njobs, u32 tile) {
    const int lane = lane_id();
    int cnt = 0;
    for (int b = 0; b < njobs; b += 64) {
        const int j = b + lane;
        const bool le = j < njobs && jobs[j].tile0 <= tile;
        cnt += (int)__popcll(__ballot(le));
    }
    return cnt - 1;
}

// A float in global memory: loads through it compile to global (not flat) loads, which
// wait on the vector memory counter only.
typedef __attribute__((address_space(1))) float gfloat;

// Value of the lane N below (row_shr) or above (row_shl) within the lane's row of 16 lanes
// (DPP, a VALU operand modifier; 0 where that lane lies outside the row).
template <int N>
__device__ inline u32 row_shr(u32 v) {
    return (u32)__builtin_amdgcn_update_dpp(0, (int)v, 0x110 + N, 0xF, 0xF, true);
}
// The two halves are shifted separately and reassembled as one register pair (a bit cast,
// not an OR of shifted halves, which the compiler would turn into two 64-bit adds).
typedef u32 u32x2 __attribute__((ext_vector_type(2)));
template <int N>
__device__ inline u64 row_shr64(u64 v) {
    const u32x2 h = __builtin_bit_cast(u32x2, v);
    u32x2 r;
    r.x = row_shr<N>(h.x);
    r.y = row_shr<N>(h.y);
    return __builtin_bit_cast(u64, r);
}
template <int N>
__device__ inline u32 row_shl(u32 v) {
    return (u32)__builtin_amdgcn_update_dpp(0, (int)v, 0x100 + N, 0xF, 0xF, true);
}

// ---------------------------------------------------------------------------
// points: per-point raycasting
// ---------------------------------------------------------------------------
// Every point of tile k owns ray slot k * kTileSimple + (its index in the tile); invalid points
// and the tail of a frame's last tile leave a hole (job kNoRay).  No counter is shared.
__global__ __launch_bounds__(256) void k_points_simple(const Job* __restrict__ jobs, int njobs,
                                                       const MapDesc* __restrict__ maps,
                                                       float4* __restrict__ rays_p,
                                                       u32* __restrict__ rays_job,
                                                       u32* __restrict__ rays_c,
                                                       JobStat* __restrict__ jst,
                                                       CallState* __restrict__ cs) {
    __shared__ u32 s_cnt[3];   // valid, invalid, out of bounds
    const int jid = job_of_tile(jobs, njobs, blockIdx.x);
    const Job J = jobs[jid];          // by value: kept in registers across the LDS atomics
    const MapDesc M = maps[J.map];
    if (threadIdx.x < 3) s_cnt[threadIdx.x] = 0;
    if (blockIdx.x == 0 && threadIdx.x == 0) cs->ray_count = gridDim.x * (u32)kTileSimple;
    __syncthreads();
    const u32 first = (blockIdx.x - J.tile0) * kTileSimple;
    u32 n_valid = 0, n_inv = 0, n_oob = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const u32 i = first + threadIdx.x + 256u * j;
        const size_t slot = (size_t)blockIdx.x * kTileSimple + threadIdx.x + 256u * j;
        u32 job = kNoRay;
        int c = -1;
        if (i < J.n) {
            const float x = J.pts[3 * (size_t)i], y = J.pts[3 * (size_t)i + 1], z = J.pts[3 * (size_t)i + 2];
            float q[3];
            c = classify_point(M, J.pose, x, y, z, q);
            if (c == 1) {
                // per-point weight: Eq. (2) 1, or the 1/z^2 factor of Eq. (5)
                const float wgt = M.weighting == 1 ? 1.0f / (z * z) : 1.0f;
                rays_p[slot] = make_float4(q[0], q[1], q[2], wgt);
                if (rays_c) rays_c[slot] = J.colors ? J.colors[i] : 0u;   // the ray's colour
                job = (u32)jid;
            }
        }
        rays_job[slot] = job;
        // per wave, from ballots
        n_valid += (u32)__popcll(__ballot(c == 1));
        n_inv += (u32)__popcll(__ballot(c == 0));
        n_oob += (u32)__popcll(__ballot(c == 2));
    }
    if (lane_id() == 0) {
        if (n_valid) atomicAdd(&s_cnt[0], n_valid);
        if (n_inv) atomicAdd(&s_cnt[1], n_inv);
        if (n_oob) atomicAdd(&s_cnt[2], n_oob);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        if (s_cnt[0]) { atomicAdd(&jst[jid].valid, (u64)s_cnt[0]); atomicAdd(&jst[jid].rays, (u64)s_cnt[0]); }
        if (s_cnt[1]) atomicAdd(&jst[jid].invalid, (u64)s_cnt[1]);
        if (s_cnt[2]) atomicAdd(&jst[jid].oob_pts, (u64)s_cnt[2]);
    }
}

// ---------------------------------------------------------------------------
// points: grouped raycasting, tile-level merge in LDS then global merge
// ---------------------------------------------------------------------------
// Fixed-point terms of one point for the exact group mean:
//   Q_k = min(rint(q_k 2^20), 2^20 - 1) with q_k = f_k - floor(f_k), f_k = p_k / v (binary32),
//   Omega = rint(w 2^wbits) (w = 1/z^2) or 1, returned as the (integral) binary32 value; it
//   is at most 2^32 (w <= 2^(32 - wbits)).
__device__ inline void group_terms(const MapDesc& M, const float q[3], float z, int g[3], u32 Q[3],
                                   float& om) {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        float f = q[k] * M.iv;
        float fl = __builtin_floorf(f);
        g[k] = (int)fl;
        float fr = f - fl;   // fl is an integer below 2^18 in magnitude: exactly (float)g[k]
        float qs = __builtin_rintf(__builtin_ldexpf(fr, 20));
        u32 Qk = (u32)qs;
        Q[k] = Qk > (1u << 20) - 1 ? (1u << 20) - 1 : Qk;
    }
    if (M.wbits > 0) {
        float w = 1.0f / (z * z);
        om = __builtin_rintf(__builtin_ldexpf(w, M.wbits));
    } else {
        om = 1.0f;
    }
}

// Inserts a (map, block) key into the per-call block set; returns its slot (0xFFFFFFFF and a
// call error when the set is full).
template <bool CHECK_FIRST>
__device__ inline u32 tset_insert(u64* tkeys, u32 tmask, u64 key, u32* tlist, u32 tlist_cap,
                                  CallState* cs) {
    u32 h = (u32)mix64(key) & tmask;
    for (u32 probe = 0; probe <= tmask; ++probe) {
        // CHECK_FIRST: a key never leaves its slot during a call, so a slot already holding it
        // needs no read-modify-write.  Where nearly every workgroup enters the same few blocks
        // (those next to a sensor), this avoids compare-and-swaps on one address, which are
        // carried out one after another; elsewhere the extra round trip costs more.  The check
        // is a device-coherent atomic load: a plain read may return a line cached before the
        // slot was cleaned by the previous call, which would let one key enter two slots.
        u64 old;
        if (CHECK_FIRST) {
            old = __hip_atomic_load(&tkeys[h], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (old == key) return h;
            if (old != kEmpty) {
                h = (h + 1) & tmask;
                continue;
            }
        }
        old = atomicCAS(&tkeys[h], kEmpty, key);
        if (old == kEmpty) {
            u32 t = atomicAdd(&cs->t_count, 1u);
            if (t < tlist_cap) { tlist[t] = h; return h; }
            cs->error = -3;   // more distinct blocks than the maps can hold
            return 0xFFFFFFFFu;
        }
        if (old == key) return h;
        h = (h + 1) & tmask;
    }
    cs->error = -3;
    return 0xFFFFFFFFu;
}

// Grouped raycasting, step 1: the points of a tile are merged by voxel (exact integer sums);
// each partial group is written as one record, tagged with the block-set slot of its voxel's
// block.  The block set is entered once per distinct block of the tile.
//
// The tile's voxel table has kTileHash slots, so that eight workgroups fit a CU.  A tile can
// have more distinct voxels than that (up to its 512 points); a run of points that finds the
// table full becomes a partial group of its own, which is exact because partial groups are
// merged again across tiles.  Table records fill the tile's record range from the front, such
// runs fill it from the back; a tile has at most kTileGrouped runs, so the two never meet.
// tile_parts holds (front count) | (back count) << 16.
constexpr int kTileHash = 256;     // voxel table slots per tile (one per thread)
constexpr int kTileBlocks = 128;   // distinct-block table slots per tile

// COLOR: the points carry colours; each partial group also sums Omega * colour per channel
// (parts_c, at the partial's index), for the group's exact mean colour.
template <bool COLOR>
__global__ __launch_bounds__(256) void k_points_grouped(const Job* __restrict__ jobs, int njobs,
                                                        const MapDesc* __restrict__ maps,
                                                        u64* __restrict__ tkeys, u32 tmask,
                                                        u32* __restrict__ tlist, u32 tlist_cap,
                                                        Partial* __restrict__ parts,
                                                        PartialColor* __restrict__ parts_c,
                                                        u32* __restrict__ tile_parts, u32 tiles_per_job,
                                                        JobStat* __restrict__ jst,
                                                        CallState* __restrict__ cs) {
    static_assert(kTileHash == 256, "one voxel slot per thread");
    constexpr int CS = COLOR ? kTileHash : 1;
    __shared__ u64 s_sc[3][CS];             // colour sums (colour calls)
    __shared__ u64 s_key[kTileHash];
    __shared__ u64 s_so[kTileHash];
    __shared__ u64 s_sq[3][kTileHash];
    __shared__ u32 s_n[kTileHash];
    __shared__ float s_pt[3][kTileHash];    // the world point of a one-point group
    __shared__ u64 s_bkey[kTileBlocks];     // distinct (map, block) keys of the tile
    __shared__ u32 s_bh[kTileBlocks];       // their block-set slots
    __shared__ u32 s_cnt[4];
    __shared__ u32 lds8[4];
    // when every frame has the same number of tiles (and there is one map), the job and map
    // follow without a dependent load
    const int jid = tiles_per_job ? (int)(blockIdx.x / tiles_per_job) : job_of_tile(jobs, njobs, blockIdx.x);
    const Job J = jobs[jid];          // by value: kept in registers across the LDS atomics
    const MapDesc M = maps[tiles_per_job ? 0u : J.map];
    s_key[threadIdx.x] = kEmpty; s_so[threadIdx.x] = 0;
    s_sq[0][threadIdx.x] = 0; s_sq[1][threadIdx.x] = 0; s_sq[2][threadIdx.x] = 0; s_n[threadIdx.x] = 0;
    if (COLOR) { s_sc[0][threadIdx.x] = 0; s_sc[1][threadIdx.x] = 0; s_sc[2][threadIdx.x] = 0; }
    if (threadIdx.x < kTileBlocks) s_bkey[threadIdx.x] = kEmpty;
    if (threadIdx.x < 4) s_cnt[threadIdx.x] = 0;
    __syncthreads();

    const u32 tile = blockIdx.x - J.tile0;
    const int lane = lane_id(), r16 = lane & 15;
    const u64 mapbits = (u64)M.map_id << 45;
    const u32 jm12 = J.jm << 12;
    Partial* const tparts = parts + (size_t)blockIdx.x * kTileGrouped;
    PartialColor* const tparts_c = COLOR ? parts_c + (size_t)blockIdx.x * kTileGrouped : nullptr;
    u32 n_valid = 0, n_inv = 0, n_oob = 0;   // per wave (from ballots)
    // both points of this thread are loaded before either is processed; a lane past the end
    // of the frame loads its first point (a frame with a tile has one) and ignores it
    u32 ii[2];
    bool inn[2];
    float px[2], py[2], pz[2];
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        if (J.width > 0) {
            const u32 tiles_x = (J.width + kTileGroupedW - 1) / kTileGroupedW;
            const u32 ty = tile / tiles_x, tx = tile - ty * tiles_x;
            const u32 col = tx * kTileGroupedW + (threadIdx.x & 31);
            const u32 row = ty * kTileGroupedH + (threadIdx.x >> 5) + 8u * j;
            inn[j] = col < J.width && (size_t)row * J.width + col < J.n;
            ii[j] = row * J.width + col;
        } else {
            ii[j] = tile * kTileGrouped + threadIdx.x + 256u * j;
            inn[j] = ii[j] < J.n;
        }
        const gfloat* src = (const gfloat*)J.pts + 3 * (size_t)(inn[j] ? ii[j] : 0u);
        px[j] = src[0]; py[j] = src[1]; pz[j] = src[2];
    }
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const bool in = inn[j];
        // this lane's contribution; a lane without a valid point gets a key no point has
        u64 key = kEmpty - 1 - (u64)lane;
        u64 so = 0, sq0 = 0, sq1 = 0, sq2 = 0;
        u64 sc0 = 0, sc1 = 0, sc2 = 0;   // Omega * colour (colour calls)
        float pw[3] = {0.f, 0.f, 0.f};
        int c = -1;
        if (in) c = classify_point(M, J.pose, px[j], py[j], pz[j], pw);
        if (c == 1) {
            int g[3];
            u32 Q[3];
            float omf;
            group_terms(M, pw, pz[j], g, Q, omf);
            key = voxel_key_of(g[0], g[1], g[2]);
            u64 om;
            if (__builtin_expect(__ballot(omf >= 0x1p32f) == 0ull, 1)) {
                // every Omega of the wave is below 2^32: 32 x 32-bit products
                const u32 o32 = (u32)omf;
                om = o32;
                sq0 = (u64)o32 * Q[0];
                sq1 = (u64)o32 * Q[1];
                sq2 = (u64)o32 * Q[2];
            } else {
                om = (u64)omf;
                sq0 = om * Q[0];
                sq1 = om * Q[1];
                sq2 = om * Q[2];
            }
            so = om;
            if (COLOR) {
                const u32 col = J.colors ? J.colors[ii[j]] : 0u;
                sc0 = om * (col & 255u);
                sc1 = om * ((col >> 8) & 255u);
                sc2 = om * ((col >> 16) & 255u);
            }
        }
        n_valid += (u32)__popcll(__ballot(c == 1));
        n_inv += (u32)__popcll(__ballot(c == 0));
        n_oob += (u32)__popcll(__ballot(c == 2));
        // Neighbouring pixels mostly share a voxel: runs of equal keys within each row of 16
        // lanes are summed first (segmented scan over DPP row shifts; integer sums, exact), so
        // only the last lane of a run enters the tile's table.  A run holds valid points only
        // (every other lane has a key of its own); its first lane is a head, found by ballot,
        // and at the step of shift N a lane adds the partial sum N lanes below when that lane
        // lies in its run (its position in the run is at least N); a step that no lane of the
        // wave needs (every run shorter than N + 1) is skipped.
        // cross-lane reads run with every lane active (never inside a short-circuit condition;
        // the skip is wave-uniform)
        const u64 prev_key = row_shr64<1>(key);
        const bool head0 = r16 == 0 || prev_key != key;
        const u64 heads = __ballot(head0);
        const u64 upto = heads & ((2ull << lane) - 1ull);     // heads at or below this lane
        const u32 runpos = (u32)lane - (u32)(63 - __clzll((long long)upto));
#define VBX_SEG_STEP(N)                                                                        \
        if (__ballot(runpos >= N) != 0ull) {                                                   \
            const u64 a_so = row_shr64<N>(so), a0 = row_shr64<N>(sq0), a1 = row_shr64<N>(sq1),  \
                      a2 = row_shr64<N>(sq2);                                                  \
            if (runpos >= N) {                                                                 \
                so += a_so; sq0 += a0; sq1 += a1; sq2 += a2;                                   \
            }                                                                                  \
            if (COLOR) {                                                                       \
                const u64 c0 = row_shr64<N>(sc0), c1 = row_shr64<N>(sc1), c2 = row_shr64<N>(sc2); \
                if (runpos >= N) { sc0 += c0; sc1 += c1; sc2 += c2; }                          \
            }                                                                                  \
        }
        VBX_SEG_STEP(1) VBX_SEG_STEP(2) VBX_SEG_STEP(4) VBX_SEG_STEP(8)
#undef VBX_SEG_STEP
        const u32 next_head = row_shl<1>((u32)head0);
        const bool tail = r16 == 15 || next_head != 0;
        const u32 cnt = runpos + 1;   // points of the run, at its last lane
        if (tail && c == 1) {
            u32 h = lds_slot<8>(key);
            bool placed = false;
            for (int probe = 0; probe < kTileHash; ++probe) {
                const u64 old = atomicCAS(&s_key[h], kEmpty, key);
                if (old == kEmpty || old == key) { placed = true; break; }
                h = (h + 1) & (kTileHash - 1);
            }
            if (placed) {
                atomicAdd(&s_so[h], so);
                atomicAdd(&s_sq[0][h], sq0);
                atomicAdd(&s_sq[1][h], sq1);
                atomicAdd(&s_sq[2][h], sq2);
                atomicAdd(&s_n[h], cnt);
                if (COLOR) { atomicAdd(&s_sc[0][h], sc0); atomicAdd(&s_sc[1][h], sc1); atomicAdd(&s_sc[2][h], sc2); }
                // read only when the group has a single point: then it is this one
                s_pt[0][h] = pw[0]; s_pt[1][h] = pw[1]; s_pt[2][h] = pw[2];
            } else {
                // the table is full: the run is written now, from the back of the tile's range,
                // and enters the block set alone
                Partial P;
                P.so_n = partial_so_n(so, cnt);
                if (cnt == 1) {
                    int g1[3];
                    u32 Q1[3];
                    float om1;
                    group_terms(M, pw, 1.0f, g1, Q1, om1);
                    pack_single(pw, Q1, P.sq);
                } else {
                    P.sq[0] = sq0; P.sq[1] = sq1; P.sq[2] = sq2;
                }
                P.h = tset_insert<false>(tkeys, tmask, mapbits | (key >> 12), tlist, tlist_cap, cs);
                P.lj = jm12 | (u32)(key & 4095u);
                const u32 idx = kTileGrouped - 1 - atomicAdd(&s_cnt[3], 1u);
                tparts[idx] = P;
                if (COLOR) tparts_c[idx] = PartialColor{{sc0, sc1, sc2}};
            }
        }
    }
    if (lane == 0) {
        if (n_valid) atomicAdd(&s_cnt[0], n_valid);
        if (n_inv) atomicAdd(&s_cnt[1], n_inv);
        if (n_oob) atomicAdd(&s_cnt[2], n_oob);
    }
    __syncthreads();

    // this thread's record: its table slot
    const int k = threadIdx.x;
    const u64 skey = s_key[k];
    const bool has_slot = skey != kEmpty;
    const u32 sn = has_slot ? s_n[k] : 0u;
    // distinct blocks of the records; a block that finds the block table full resolves alone
    const u64 bk = mapbits | (skey >> 12);
    u32 bh = 0xFFFFFFFFu;   // block table slot
    if (has_slot) {
        u32 b = lds_slot<7>(bk);
        for (int probe = 0; probe < kTileBlocks; ++probe) {
            const u64 old = atomicCAS(&s_bkey[b], kEmpty, bk);
            if (old == kEmpty || old == bk) { bh = b; break; }
            b = (b + 1) & (kTileBlocks - 1);
        }
    }
    const bool direct = has_slot && bh == 0xFFFFFFFFu;
    // table records of tile k take slots [k * kTileGrouped, k * kTileGrouped + count): a tile has
    // at most kTileGrouped points, so the slots never overlap and no counter is shared
    u32 tot;
    const u32 incl = block_count_256(has_slot, lds8, &tot);
    if (threadIdx.x < kTileBlocks) {
        const u64 tb = s_bkey[threadIdx.x];
        if (tb != kEmpty) s_bh[threadIdx.x] = tset_insert<false>(tkeys, tmask, tb, tlist, tlist_cap, cs);
    }
    const u32 hdirect = direct ? tset_insert<false>(tkeys, tmask, bk, tlist, tlist_cap, cs) : 0xFFFFFFFFu;
    __syncthreads();
    if (threadIdx.x == 0) tile_parts[blockIdx.x] = tot | (s_cnt[3] << 16);
    if (has_slot) {
        Partial P;
        P.so_n = partial_so_n(s_so[k], sn);
        if (sn == 1) {
            // the world point as it was grouped, and its Q_k
            const float p1[3] = {s_pt[0][k], s_pt[1][k], s_pt[2][k]};
            int g1[3];
            u32 Q1[3];
            float om1;
            group_terms(M, p1, 1.0f, g1, Q1, om1);
            pack_single(p1, Q1, P.sq);
        } else {
            P.sq[0] = s_sq[0][k]; P.sq[1] = s_sq[1][k]; P.sq[2] = s_sq[2][k];
        }
        P.h = direct ? hdirect : s_bh[bh];
        P.lj = jm12 | (u32)(skey & 4095u);
        tparts[incl - 1] = P;
        if (COLOR) tparts_c[incl - 1] = PartialColor{{s_sc[0][k], s_sc[1][k], s_sc[2][k]}};
    }
    if (threadIdx.x == 0) {
        if (s_cnt[0]) atomicAdd(&jst[jid].valid, (u64)s_cnt[0]);
        if (s_cnt[1]) atomicAdd(&jst[jid].invalid, (u64)s_cnt[1]);
        if (s_cnt[2]) atomicAdd(&jst[jid].oob_pts, (u64)s_cnt[2]);
    }
}

template __global__ void k_points_grouped<false>(const Job*, int, const MapDesc*, u64*, u32, u32*, u32, Partial*,
                                                 PartialColor*, u32*, u32, JobStat*, CallState*);
template __global__ void k_points_grouped<true>(const Job*, int, const MapDesc*, u64*, u32, u32*, u32, Partial*,
                                                PartialColor*, u32*, u32, JobStat*, CallState*);

// Dense index of every block-set entry listed so far (its list position).
__global__ __launch_bounds__(256) void k_densify(const u32* __restrict__ tlist, u32 tlist_cap,
                                                 u32* __restrict__ tval,
                                                 const CallState* __restrict__ cs) {
    const u32 nt = cs->error ? 0u : (cs->t_count < tlist_cap ? cs->t_count : tlist_cap);
    for (u32 i = blockIdx.x * 256u + threadIdx.x; i < nt; i += gridDim.x * 256u) tval[tlist[i]] = i;
}

// Grouped raycasting, step 2: counting sort of the partial groups by (block, frame).  One
// wave takes tpw (1 or 2) consecutive tiles and walks their partials as one list (the first
// tile's, then the second's), two records per lane at a time, so that the loads and atomics of
// up to 128 records are in flight together.  Two tiles per wave pay where the tiles outnumber
// the waves the chip holds; with fewer tiles, one per wave keeps more waves running.

// Sort bin of a partial group: (block t, frame, eighth of the block's voxels), JM frames per
// block, so that a bin spans at most kMergeVox distinct voxels.
__device__ inline u32 group_bin(u32 t, u32 lj, u32 JM) {
    return (t * JM + (lj >> 12)) * (u32)kGroupSubBins + (lj & 4095u) / (4096u / (u32)kGroupSubBins);
}

// Position of a tile's i-th record, i < np: nf records at the front of its range, the other
// np - nf at the back.
__device__ inline u32 tile_record(u32 i, u32 nf, u32 np) {
    return i < nf ? i : (u32)kTileGrouped - np + i;
}

// The records of tile tile0 and, when tpw is 2 and it exists, of tile0 + 1, as one list.
struct TilePair {
    u32 tile0, nf0, np0, nf1, np1;
    __device__ TilePair(const u32* tile_parts, u32 ntiles, u32 t0, u32 tpw) : tile0(t0) {
        const u32 a = tile_parts[t0];
        const u32 b = tpw == 2u && t0 + 1u < ntiles ? tile_parts[t0 + 1u] : 0u;
        nf0 = a & 0xFFFFu; np0 = nf0 + (a >> 16);
        nf1 = b & 0xFFFFu; np1 = nf1 + (b >> 16);
    }
    __device__ u32 count() const { return np0 + np1; }
    // index in the partial array of record r < count()
    __device__ size_t record(u32 r) const {
        return r < np0 ? (size_t)tile0 * kTileGrouped + tile_record(r, nf0, np0)
                       : (size_t)(tile0 + 1u) * kTileGrouped + tile_record(r - np0, nf1, np1);
    }
};

__global__ __launch_bounds__(256) void k_gbin_count(const Partial* __restrict__ parts,
                                                    const u32* __restrict__ tile_parts, u32 ntiles,
                                                    const u32* __restrict__ tval,
                                                    u32* __restrict__ bins, u32 JM, u32 tpw,
                                                    const CallState* __restrict__ cs) {
    if (cs->error) return;
    const u32 tile0 = (blockIdx.x * 4u + (threadIdx.x >> 6)) * tpw;
    if (tile0 >= ntiles) return;   // whole wave
    const u32 lane = (u32)lane_id();
    const TilePair tp(tile_parts, ntiles, tile0, tpw);
    const u32 np = tp.count();
    for (u32 b0 = 0; b0 < np; b0 += 128) {
        const u32 r0 = b0 + lane, r1 = r0 + 64u;
        const bool a0 = r0 < np, a1 = r1 < np;
        u32 h0 = 0, l0 = 0, h1 = 0, l1 = 0;
        if (a0) { const Partial& P = parts[tp.record(r0)]; h0 = P.h; l0 = P.lj; }
        if (a1) { const Partial& P = parts[tp.record(r1)]; h1 = P.h; l1 = P.lj; }
        // both dense indices loaded together (an inactive lane reads entry 0 and ignores it)
        const u32 t0 = tval[h0], t1 = tval[h1];
        const u32 k0 = a0 ? group_bin(t0, l0, JM) : 0u;
        const u32 k1 = a1 ? group_bin(t1, l1, JM) : 0u;
        wave_count_by_key(bins, a0, k0);
        wave_count_by_key(bins, a1, k1);
    }
}

__global__ __launch_bounds__(256) void k_gscatter(const Partial* __restrict__ parts,
                                                  const u32* __restrict__ tile_parts, u32 ntiles,
                                                  const u32* __restrict__ tval,
                                                  u32* __restrict__ bins, const u32* __restrict__ off,
                                                  u32 JM, u32 tpw, Partial* __restrict__ sorted,
                                                  const PartialColor* __restrict__ parts_c,
                                                  PartialColor* __restrict__ sorted_c,
                                                  const CallState* __restrict__ cs) {
    if (cs->error) return;
    const u32 tile0 = (blockIdx.x * 4u + (threadIdx.x >> 6)) * tpw;
    if (tile0 >= ntiles) return;   // whole wave
    const u32 lane = (u32)lane_id();
    const TilePair tp(tile_parts, ntiles, tile0, tpw);
    const u32 np = tp.count();
    for (u32 b0 = 0; b0 < np; b0 += 128) {
        const u32 r0 = b0 + lane, r1 = r0 + 64u;
        const bool a[2] = {r0 < np, r1 < np};
        Partial P0, P1;
        if (a[0]) P0 = parts[tp.record(r0)];
        if (a[1]) P1 = parts[tp.record(r1)];
        // both dense indices loaded together (an inactive lane reads entry 0 and ignores it)
        const u32 t0 = tval[a[0] ? P0.h : 0u], t1 = tval[a[1] ? P1.h : 0u];
        const u32 k[2] = {a[0] ? group_bin(t0, P0.lj, JM) : 0u, a[1] ? group_bin(t1, P1.lj, JM) : 0u};
        u32 pos[2];
        wave_claim_by_keys<2>(bins, off, a, k, pos);
        if (a[0]) sorted[pos[0]] = P0;
        if (a[1]) sorted[pos[1]] = P1;
        if (parts_c) {
            if (a[0]) sorted_c[pos[0]] = parts_c[tp.record(r0)];
            if (a[1]) sorted_c[pos[1]] = parts_c[tp.record(r1)];
        }
    }
}

// Grouped raycasting, step 3: merging the partial groups of each sort bin (block, frame,
// eighth of the block's voxels; JMS bins per block) by voxel and casting one ray per group --
// the exact weighted mean (a group of one point keeps the point) with the group's summed weight.
//
// Work is cut into chunks of kMergeSpan consecutive sorted partials; a chunk owns the bins
// whose first partial falls in it.  Consecutive bins of a chunk are merged together in one
// LDS hash keyed by (bin in batch, local voxel) while they hold at most kMergeBatch partials;
// a bin larger than that is merged alone, in one pass over a dense table of its kMergeVox
// voxels.
// The rays of bin b take slots [off[b], off[b] + groups) and the rest of its range is marked
// empty, so no counter is shared between workgroups.
constexpr int kMergeVox = 2 * kMergeSpan;        // LDS table entries (hash slots or dense voxels)
constexpr int kMergeBatch = kMergeSpan * 5 / 4;  // partials merged in one hash pass (load <= 0.625)
constexpr int kMergePerThread = kMergeVox / 256;
static_assert(kGroupSubBins * kMergeVox == 4096 && kMergePerThread * 256 == kMergeVox, "merge table");

// Ray of a merged group: towards its single point, else towards the exact weighted mean,
// carrying the group's summed weight.
__device__ inline void group_ray(const MapDesc& M, int bx, int by, int bz, u32 l, u32 n, u64 so,
                                 const u64* sq, const u32* hi, const float* p1, float4& ray) {
    const int g[3] = {16 * bx + (int)(l & 15), 16 * by + (int)((l >> 4) & 15), 16 * bz + (int)(l >> 8)};
    float p[3];
    if (n == 1) {
        p[0] = p1[0]; p[1] = p1[1]; p[2] = p1[2];
    } else {
        const double den = (double)so * 1048576.0;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const double m = ((double)(u64)hi[k] * 18446744073709551616.0 + (double)sq[k]) / den;
            p[k] = (float)(((double)g[k] + m) * (double)M.v);
        }
    }
    const float wgt = M.wbits > 0 ? (float)((double)so * __builtin_ldexp(1.0, -M.wbits)) : (float)n;
    ray = make_float4(p[0], p[1], p[2], wgt);
}

// Sums a partial group into merge slot v: a one-point partial contributes weight * Q_k.
__device__ inline void merge_partial(const Partial& P, u32 v, u64* m_so, u64 (*m_sq)[kMergeVox],
                                     u32 (*m_hi)[kMergeVox], u32* m_n, float (*m_p)[kMergeVox]) {
    u64 add[3] = {P.sq[0], P.sq[1], P.sq[2]};
    const u64 so = partial_so(P.so_n);
    const u32 n = partial_n(P.so_n);
    if (n == 1) {
        float p1[3];
        u32 Q[3];
        unpack_single(P.sq, p1, Q);
        add[0] = so * Q[0];
        add[1] = so * Q[1];
        add[2] = so * Q[2];
        m_p[0][v] = p1[0]; m_p[1][v] = p1[1]; m_p[2][v] = p1[2];   // read only if the group stays single
    }
    // the three returning adds are issued together, their carries (rare) added afterwards
    u64 old[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) old[k] = atomicAdd(&m_sq[k][v], add[k]);
    atomicAdd(&m_so[v], so);
    atomicAdd(&m_n[v], n);
    bool carry[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) carry[k] = old[k] + add[k] < old[k];
    if (__builtin_expect(__ballot(carry[0] | carry[1] | carry[2]) != 0ull, 0)) {
#pragma unroll
        for (int k = 0; k < 3; ++k)
            if (carry[k]) atomicAdd(&m_hi[k][v], 1u);
    }
}

// The mean colour of a group, per channel round(sc / so) to nearest with ties to even, in
// integer arithmetic (the same rounding as the position mean's: no binary floating point).
__device__ inline u32 group_color(const u64 sc[3], u64 so) {
    u32 c = 0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const u64 q = sc[k] / so, r = sc[k] - q * so;
        const u64 v = q + ((2 * r > so || (2 * r == so && (q & 1))) ? 1u : 0u);
        c |= (u32)(v > 255u ? 255u : v) << (8 * k);
    }
    return c;
}

template <bool COLOR>
__global__ __launch_bounds__(256) void k_group_merge(const Job* __restrict__ jobs,
                                                     const MapDesc* __restrict__ maps,
                                                     const u64* __restrict__ tkeys,
                                                     const u32* __restrict__ tlist,
                                                     const u32* __restrict__ off,
                                                     const u32* __restrict__ chunk_first,
                                                     const Partial* __restrict__ sorted, u32 JMS,
                                                     const PartialColor* __restrict__ sorted_c,
                                                     float4* __restrict__ rays_p,
                                                     u32* __restrict__ rays_job,
                                                     u32* __restrict__ rays_c,
                                                     JobStat* __restrict__ jst,
                                                     CallState* __restrict__ cs) {
    constexpr int CV = COLOR ? kMergeVox : 1;
    __shared__ u64 m_sc[3][CV];        // colour sums (colour calls)
    __shared__ u32 m_key[kMergeVox];   // hash: (bin in batch << 12 | local) + 1, 0 = free
    __shared__ u64 m_so[kMergeVox];
    __shared__ u64 m_sq[3][kMergeVox];
    __shared__ u32 m_hi[3][kMergeVox];
    __shared__ u32 m_n[kMergeVox];
    __shared__ float m_p[3][kMergeVox];   // the point of a one-point group
    __shared__ u32 s_nr[kMergeBatch];  // rays emitted per bin of the batch
    __shared__ u32 s_off[kMergeBatch + 2];
    __shared__ u64 s_tk[kMergeBatch];  // block-set key of each bin's block
    __shared__ u32 lds8[4];
    for (int i = threadIdx.x; i < kMergeVox; i += 256) {
        m_key[i] = 0; m_so[i] = 0; m_sq[0][i] = 0; m_sq[1][i] = 0; m_sq[2][i] = 0;
        m_hi[0][i] = 0; m_hi[1][i] = 0; m_hi[2][i] = 0; m_n[i] = 0;
        if (COLOR) { m_sc[0][i] = 0; m_sc[1][i] = 0; m_sc[2][i] = 0; }
    }
    const u32 nb = cs->error ? 0u : cs->t_count * JMS;
    const u32 total = nb ? off[nb] : 0u;
    if (blockIdx.x == 0 && threadIdx.x == 0) cs->ray_count = total;
    const u32 nchunks = (total + kMergeSpan - 1) / kMergeSpan;
    // The workgroup takes chunks blockIdx.x, blockIdx.x + gridDim.x, ...; each iteration below
    // merges one batch (or one large bin) of its current chunk.  The next batch's bin offsets,
    // block keys and first partials are loaded while the current one is merged, so that their
    // latency overlaps the merge instead of preceding it.
    // (c, b, be): chunk, first bin of the batch, end of the chunk's bins; a chunk that owns no
    // bin (a large bin started in an earlier chunk) is passed over.
    auto seek = [&](u32& c_, u32& b_, u32& be_) {
        for (; c_ < nchunks; c_ += gridDim.x) {
            b_ = chunk_first[c_];
            be_ = c_ + 1 < nchunks ? chunk_first[c_ + 1] : nb;
            if (b_ < be_) return;
        }
    };
    // loads of the batch at (b_, be_), in two steps (the second needs the first's values):
    // this thread's bins k = threadIdx.x and k + 256 (offsets, then block keys through the
    // block list), and the batch's partials at positions threadIdx.x and threadIdx.x + 256
    u32 nx_off[2] = {0u, 0u}, nx_tl[2] = {0u, 0u}, nx_p0 = 0u;
    u64 nx_tk[2] = {0ull, 0ull};
    Partial nx_P[2] = {};
    auto load_offsets = [&](u32 b_, u32 be_) {
        const u32 wn_ = be_ - b_ < (u32)kMergeBatch ? be_ - b_ : (u32)kMergeBatch;
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const u32 k = threadIdx.x + 256u * (u32)q;
            if (k <= wn_) nx_off[q] = off[b_ + k];
            if (k < wn_) nx_tl[q] = tlist[(b_ + k) / JMS];
        }
        nx_p0 = off[b_];   // the batch's first partial (the same address in every thread)
    };
    auto load_rest = [&](u32 b_, u32 be_) {
        const u32 wn_ = be_ - b_ < (u32)kMergeBatch ? be_ - b_ : (u32)kMergeBatch;
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const u32 k = threadIdx.x + 256u * (u32)q;
            if (k < wn_) nx_tk[q] = tkeys[nx_tl[q]];
            // (a hash batch holds at most kMergeBatch partials: none is loaded beyond them)
            const u32 e = nx_p0 + threadIdx.x + 256u * (u32)q;
            if (e < total && e < nx_p0 + (u32)kMergeBatch) nx_P[q] = sorted[e];
        }
    };
    u32 c = blockIdx.x, b = 0, be = 0;
    seek(c, b, be);
    if (c < nchunks) {
        load_offsets(b, be);
        load_rest(b, be);
    }
    __syncthreads();
    while (c < nchunks) {
        // stage the offsets and block keys of up to kMergeBatch bins
        const u32 wn = be - b < (u32)kMergeBatch ? be - b : (u32)kMergeBatch;
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const u32 k = threadIdx.x + 256u * (u32)q;
            if (k <= wn) s_off[k] = nx_off[q];
            if (k < wn) s_tk[k] = nx_tk[q];
        }
        const Partial cur_P[2] = {nx_P[0], nx_P[1]};
        // the partial at position e, the it-th of this thread (loaded ahead when it lies among
        // the batch's first kMergeBatch partials)
        auto partial_at = [&](u32 e, u32 it) {
            Partial P;
            if (it == 0u) P = cur_P[0];
            else if (it == 1u && e < s_off[0] + (u32)kMergeBatch) P = cur_P[1];
            else P = sorted[e];
            return P;
        };
        __syncthreads();
        const u32 base = s_off[0];
        // bins [b, b + nbat) hold at most kMergeBatch partials: nbat is the largest n <= wn
        // with s_off[n] - base <= kMergeBatch (offsets are non-decreasing)
        u32 nbat = 0;
        {
            u32 lo_n = 0, hi_n = wn;
            while (lo_n < hi_n) {
                const u32 mid = (lo_n + hi_n + 1) >> 1;
                if (s_off[mid] - base <= (u32)kMergeBatch) lo_n = mid; else hi_n = mid - 1;
            }
            nbat = lo_n;
        }
        // the next batch: the bins after this one in the chunk, else the next chunk's
        u32 c_n = c, b_n = b + (nbat ? nbat : 1u), be_n = be;
        if (b_n >= be_n) {
            c_n += gridDim.x;
            seek(c_n, b_n, be_n);
        }
        const bool more = c_n < nchunks;
        if (nbat == 0) {
            // ---- a bin too large for one hash pass: its at most kMergeVox voxels (one
            // eighth of the block) over a dense table
            const u32 lo = s_off[0], hi = s_off[1];
            const u32 t = b / JMS, rb = b - t * JMS;
            const u32 jm = rb / (u32)kGroupSubBins, qd = rb % (u32)kGroupSubBins;
            const u64 tk = s_tk[0];
            const MapDesc& M = maps[(u32)(tk >> 45)];
            const int jid = M.job0 + (int)jm;
            int bx, by, bz;
            unpack_block(tk & ((1ull << 45) - 1), bx, by, bz);
            u32 it = 0;
            for (u32 e = lo + threadIdx.x; e < hi; e += 256, ++it) {
                const Partial P = partial_at(e, it);
                const u32 vv = P.lj & (u32)(kMergeVox - 1);
                merge_partial(P, vv, m_so, m_sq, m_hi, m_n, m_p);
                if (COLOR)
                    for (int k = 0; k < 3; ++k) atomicAdd(&m_sc[k][vv], sorted_c[e].sc[k]);
            }
            if (more) load_offsets(b_n, be_n);
            __syncthreads();
            float4 ray[kMergePerThread];
            u32 rcol[kMergePerThread];
            bool has[kMergePerThread];
            u32 nmine = 0;
#pragma unroll
            for (int r = 0; r < kMergePerThread; ++r) {
                const int v = threadIdx.x + 256 * r;
                const u32 n = m_n[v];
                has[r] = n != 0;
                ray[r] = make_float4(0.f, 0.f, 0.f, 0.f);
                if (!n) continue;
                const u64 sq[3] = {m_sq[0][v], m_sq[1][v], m_sq[2][v]};
                const u32 hw[3] = {m_hi[0][v], m_hi[1][v], m_hi[2][v]};
                const float p1[3] = {m_p[0][v], m_p[1][v], m_p[2][v]};
                group_ray(M, bx, by, bz, qd * (u32)kMergeVox + (u32)v, n, m_so[v], sq, hw, p1, ray[r]);
                rcol[r] = 0u;
                if (COLOR) {
                    const u64 sc[3] = {m_sc[0][v], m_sc[1][v], m_sc[2][v]};
                    rcol[r] = group_color(sc, m_so[v]);
                    m_sc[0][v] = 0; m_sc[1][v] = 0; m_sc[2][v] = 0;
                }
                nmine++;
                m_so[v] = 0; m_sq[0][v] = 0; m_sq[1][v] = 0; m_sq[2][v] = 0;
                m_hi[0][v] = 0; m_hi[1][v] = 0; m_hi[2][v] = 0; m_n[v] = 0;
            }
            u32 nrays;
            const u32 incl = block_scan_256(nmine, lds8, &nrays);
            u32 pos = lo + incl - nmine;
#pragma unroll
            for (int r = 0; r < kMergePerThread; ++r) {
                if (!has[r]) continue;
                rays_p[pos] = ray[r];
                rays_job[pos] = (u32)jid;
                if (COLOR) rays_c[pos] = rcol[r];
                pos++;
            }
            if (more) load_rest(b_n, be_n);
            for (u32 e = lo + nrays + threadIdx.x; e < hi; e += 256) rays_job[e] = kNoRay;
            if (threadIdx.x == 0 && nrays) atomicAdd(&jst[jid].rays, (u64)nrays);
            __syncthreads();
        } else {
            // ---- hash merge of bins [b, b + nbat)
            const u32 pend = s_off[nbat];
            for (u32 k = threadIdx.x; k < nbat; k += 256) s_nr[k] = 0;
            __syncthreads();
            u32 it = 0;
            for (u32 e = base + threadIdx.x; e < pend; e += 256, ++it) {
                const Partial P = partial_at(e, it);
                // bin of partial e: the last staged bin whose start is <= e
                u32 lo_i = 0, hi_i = nbat - 1;
                while (lo_i < hi_i) {
                    const u32 mid = (lo_i + hi_i + 1) >> 1;
                    if (s_off[mid] <= e) lo_i = mid; else hi_i = mid - 1;
                }
                const u32 key = ((lo_i << 12) | (P.lj & 4095u)) + 1u;
                u32 h = (u32)mix64(key) & (kMergeVox - 1);
                for (;;) {
                    const u32 old = atomicCAS(&m_key[h], 0u, key);
                    if (old == 0u || old == key) break;
                    h = (h + 1) & (kMergeVox - 1);
                }
                merge_partial(P, h, m_so, m_sq, m_hi, m_n, m_p);
                if (COLOR)
                    for (int k = 0; k < 3; ++k) atomicAdd(&m_sc[k][h], sorted_c[e].sc[k]);
            }
            if (more) load_offsets(b_n, be_n);
            __syncthreads();
            for (int h = threadIdx.x; h < kMergeVox; h += 256) {
                const u32 key = m_key[h];
                if (!key) continue;
                const u32 bi = (key - 1u) >> 12, l = (key - 1u) & 4095u;
                const u32 bb = b + bi;
                const u32 t = bb / JMS, jm = (bb - t * JMS) / (u32)kGroupSubBins;
                const u64 tk = s_tk[bi];
                const MapDesc& M = maps[(u32)(tk >> 45)];
                const int jid = M.job0 + (int)jm;
                int bx, by, bz;
                unpack_block(tk & ((1ull << 45) - 1), bx, by, bz);
                const u64 sq[3] = {m_sq[0][h], m_sq[1][h], m_sq[2][h]};
                const u32 hw[3] = {m_hi[0][h], m_hi[1][h], m_hi[2][h]};
                const float p1[3] = {m_p[0][h], m_p[1][h], m_p[2][h]};
                float4 ray;
                group_ray(M, bx, by, bz, l, m_n[h], m_so[h], sq, hw, p1, ray);
                const u32 pos = s_off[bi] + atomicAdd(&s_nr[bi], 1u);
                rays_p[pos] = ray;
                rays_job[pos] = (u32)jid;
                if (COLOR) {
                    const u64 sc[3] = {m_sc[0][h], m_sc[1][h], m_sc[2][h]};
                    rays_c[pos] = group_color(sc, m_so[h]);
                    m_sc[0][h] = 0; m_sc[1][h] = 0; m_sc[2][h] = 0;
                }
                m_key[h] = 0; m_so[h] = 0; m_sq[0][h] = 0; m_sq[1][h] = 0; m_sq[2][h] = 0;
                m_hi[0][h] = 0; m_hi[1][h] = 0; m_hi[2][h] = 0; m_n[h] = 0;
            }
            if (more) load_rest(b_n, be_n);
            __syncthreads();
            // empty slots of each bin, and per-frame ray counts (one thread per bin)
            for (u32 k = threadIdx.x; k < nbat; k += 256) {
                const u32 nr = s_nr[k];
                for (u32 e = s_off[k] + nr; e < s_off[k + 1]; ++e) rays_job[e] = kNoRay;
                if (nr) {
                    const u32 bb = b + k;
                    const u32 t = bb / JMS;
                    const MapDesc& M = maps[(u32)(s_tk[k] >> 45)];
                    atomicAdd(&jst[M.job0 + (bb - t * JMS) / (u32)kGroupSubBins].rays, (u64)nr);
                }
            }
            __syncthreads();
        }
        c = c_n; b = b_n; be = be_n;
    }
}
template __global__ void k_group_merge<false>(const Job*, const MapDesc*, const u64*, const u32*, const u32*,
                                              const u32*, const Partial*, u32, const PartialColor*, float4*, u32*,
                                              u32*, JobStat*, CallState*);
template __global__ void k_group_merge<true>(const Job*, const MapDesc*, const u64*, const u32*, const u32*,
                                             const u32*, const Partial*, u32, const PartialColor*, float4*, u32*,
                                             u32*, JobStat*, CallState*);

// ---------------------------------------------------------------------------
// cross: walk the band of each ray, record (block, ray) crossings
// ---------------------------------------------------------------------------
// A workgroup takes a contiguous range of ray slots, 256 at a time, in three phases separated
// by barriers:
//  1. find the blocks of every ray's band and enter their keys in the workgroup's LDS set;
//  2. enter each key new to the set in the per-call block set (global);
//  3. write ray i's crossings (block-set slots) to cross[i * MB + c].
// The LDS set is kept from one batch of rays to the next, so a block that consecutive rays
// share (they come sorted by block, or in sensor order) enters the global set once per
// workgroup rather than once per batch.
constexpr int kCrossSlots = 2048;   // LDS block-key set
constexpr int kCrossBatchKeys = 256 * 7;   // keys one batch can add (256 rays x 7 blocks)
constexpr u32 kCrossPending = 0xFFFFFFFEu; // an LDS set entry not yet in the global set

// Enters key in the LDS set; returns its slot, with *added when this call put it there.
__device__ inline u32 lds_set_insert(u64* keys, u64 key, bool* added) {
    static_assert(kCrossSlots == 2048, "slot hash bits");
    u32 h = lds_slot<11>(key);
    for (;;) {
        const u64 old = atomicCAS(&keys[h], kEmpty, key);
        if (old == kEmpty || old == key) {
            *added = old == kEmpty;
            return h;
        }
        h = (h + 1) & (kCrossSlots - 1);
    }
}

// A ray crosses at most 7 blocks (the band is at most 28 voxels long): the LDS set slots of
// its blocks, 16 bits each, fit two 64-bit registers.
constexpr u32 kCrossHeld = 8;

__global__ __launch_bounds__(256) void k_cross(const Job* __restrict__ jobs,
                                               const MapDesc* __restrict__ maps,
                                               const float4* __restrict__ rays_p,
                                               const u32* __restrict__ rays_job,
                                               u64* __restrict__ tkeys, u32 tmask,
                                               u32* __restrict__ tlist, u32 tlist_cap,
                                               u32* __restrict__ cross, unsigned char* __restrict__ ncross,
                                               u32 MB, u32* __restrict__ hbins, u32 JM,
                                               JobStat* __restrict__ jst,
                                               CallState* __restrict__ cs, u32 ray_cap) {
    __shared__ u64 s_key[kCrossSlots];
    __shared__ u32 s_h[kCrossSlots];   // global block-set slot of each key (kCrossPending: not yet)
    __shared__ u32 s_pend[kCrossSlots / 32];   // bit per slot: a key new to the set this batch
    __shared__ u32 s_fill;             // keys in the LDS set
    const u32 nrays = cs->ray_count < ray_cap ? cs->ray_count : ray_cap;
    const u32 nbatch = (nrays + 255u) / 256u;
    const u32 per = (nbatch + gridDim.x - 1u) / gridDim.x;
    const u32 bt0 = blockIdx.x * per;
    const u32 bt1 = bt0 + per < nbatch ? bt0 + per : nbatch;
    for (int k = threadIdx.x; k < kCrossSlots; k += 256) s_key[k] = kEmpty;
    for (int k = threadIdx.x; k < kCrossSlots / 32; k += 256) s_pend[k] = 0;
    if (threadIdx.x == 0) s_fill = 0;
    __syncthreads();
    // the first batch's ray slots; each batch loads the next one's while it works
    u32 nxt_job = kNoRay;
    float4 nxt_p = make_float4(0.f, 0.f, 0.f, 0.f);
    if (bt0 < bt1 && bt0 * 256u + threadIdx.x < nrays) {
        nxt_job = rays_job[bt0 * 256u + threadIdx.x];
        nxt_p = rays_p[bt0 * 256u + threadIdx.x];   // an empty slot's point is loaded and ignored
    }
    for (u32 bt = bt0; bt < bt1; ++bt) {
        // a batch adds at most kCrossBatchKeys keys: the set is emptied before it could overflow
        // (s_fill is read by every thread before the barrier, and changed only after it)
        if (s_fill > (u32)(kCrossSlots - kCrossBatchKeys)) {
            __syncthreads();
            for (int k = threadIdx.x; k < kCrossSlots; k += 256) s_key[k] = kEmpty;
            if (threadIdx.x == 0) s_fill = 0;
            __syncthreads();
        }
        const u32 i = bt * 256u + threadIdx.x;
        bool ok = false;
        const u32 jid = nxt_job;
        const bool live = i < nrays && jid != kNoRay;
        const float4 rp = nxt_p;
        nxt_job = kNoRay;
        if (bt + 1u < bt1 && i + 256u < nrays) {
            nxt_job = rays_job[i + 256u];
            nxt_p = rays_p[i + 256u];
        }
        float p[3] = {rp.x, rp.y, rp.z}, s[3] = {0.f, 0.f, 0.f};
        u64 mapbits = 0;
        u64 held0 = 0, held1 = 0;   // LDS set slots of the crossed blocks, in crossing order
        u32 nc = 0, added = 0, jm = 0;
        const MapDesc* Mp = maps;
        if (live) {
            const Job& J = jobs[jid];
            Mp = &maps[J.map];
            jm = J.jm;
            s[0] = J.pose[3]; s[1] = J.pose[7]; s[2] = J.pose[11];
            mapbits = (u64)Mp->map_id << 45;
            float e[3], r;
            Walk w;
            ok = walk_setup(*Mp, p, s, e, r, w);
            // phase 1: the blocks the band enters, in walk order.  They follow from the walk's
            // block-changing steps alone (every 16th step of an axis), with the crossing
            // parameters of the voxel walk, which is not stepped here.
            if (ok) {
                BlockWalk bw;
                block_walk_init(w, bw);
                // (the walk's form is uniform across the workgroup's map: two loops, no branch
                // inside either)
                if (Mp->full_ray != 0) {
                    for (int guard = 0, axis = 0; axis >= 0 && guard <= Mp->max_steps;
                         ++guard, axis = block_walk_next(bw)) {
                        const u64 bk = pack_block(bw.b[0], bw.b[1], bw.b[2]);
                        // a whole ray crosses up to MB blocks, more than the LDS set and
                        // registers hold: each crossing enters the call's block set at once
                        const u32 h = tset_insert<true>(tkeys, tmask, mapbits | bk, tlist, tlist_cap, cs);
                        if (nc < MB) cross[(size_t)i * MB + nc] = h;
                        // (a failed insert is an error of the call and is not counted)
                        if (hbins) wave_count_by_key(hbins, nc < MB && h != 0xFFFFFFFFu, h * JM + jm);
                        nc++;
                    }
                } else {
                    for (int guard = 0, axis = 0; axis >= 0 && guard <= Mp->max_steps;
                         ++guard, axis = block_walk_next(bw)) {
                        const u64 bk = pack_block(bw.b[0], bw.b[1], bw.b[2]);
                        bool fresh;
                        const u32 h = lds_set_insert(s_key, mapbits | bk, &fresh);
                        if (fresh) {
                            s_h[h] = kCrossPending;
                            atomicOr(&s_pend[h >> 5], 1u << (h & 31u));
                            added++;
                        }
                        // slot c of the crossing in held0 (c < 4) or held1 (4 <= c < 8)
                        const u64 sh = (u64)h << (16u * (nc & 3u));
                        held0 |= nc < 4u ? sh : 0ull;
                        held1 |= (nc >= 4u && nc < kCrossHeld) ? sh : 0ull;
                        nc++;
                    }
                }
            }
        }
        {
            const u32 wa = wave_sum(added);
            if (lane_id() == 0 && wa) atomicAdd(&s_fill, wa);
        }
        __syncthreads();
        // phase 2: each block new to the LDS set enters the per-call block set (the slots
        // marked in s_pend, a word of 32 per thread; the marks are cleared for the next batch)
        for (int k = threadIdx.x; k < kCrossSlots / 32; k += 256) {
            u32 bits = s_pend[k];
            if (bits) {
                s_pend[k] = 0;
                while (bits) {
                    const u32 slot = (u32)k * 32u + (u32)(__ffs(bits) - 1);
                    bits &= bits - 1u;
                    s_h[slot] = tset_insert<true>(tkeys, tmask, s_key[slot], tlist, tlist_cap, cs);
                }
            }
        }
        __syncthreads();
        // phase 3: crossing c of ray slot i goes to cross[i * MB + c], and (raycasting calls)
        // counts towards its (block-set slot, frame) bin
        u32 nband = 0;   // band crossings, whose slots are held in registers
        if (i < nrays) {
            const bool full = live && Mp->full_ray != 0;
            if (nc > MB || (!full && nc > kCrossHeld)) {   // cannot happen: MB bounds the walk
                cs->error = -4;
                nc = 0;
            }
            if (!full) {
                nband = nc;
                for (u32 c = 0; c < nc; ++c)
                    cross[(size_t)i * MB + c] = s_h[(u32)((c < 4 ? held0 : held1) >> (16 * (c & 3))) & 0xFFFFu];
            }
            ncross[i] = (unsigned char)nc;
        }
        if (hbins) {
            for (u32 c = 0; c < kCrossHeld; ++c) {
                if (__ballot(c < nband) == 0ull) break;
                const u32 h = c < nband ? s_h[(u32)((c < 4 ? held0 : held1) >> (16 * (c & 3))) & 0xFFFFu]
                                        : 0xFFFFFFFFu;
                const bool act = h != 0xFFFFFFFFu;   // a failed insert is an error of the call
                wave_count_by_key(hbins, act, act ? h * JM + jm : 0u);
            }
        }
        // out-of-bounds rays per frame (rare); rays were counted when created
        const bool oob = live && !ok;
        u64 pending = __ballot(oob);
        const int lane = lane_id();
        while (pending) {
            int leader = __ffsll((long long)pending) - 1;
            u32 k = __shfl(jid, leader);
            u64 grp = __ballot(((pending >> lane) & 1ull) && jid == k);
            if (lane == leader) atomicAdd(&jst[k].oob_rays, (u64)__popcll(grp));
            pending &= ~grp;
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// resolve / commit: wavefront-cooperative probing of the map's block hash
// ---------------------------------------------------------------------------
// Wavefront-cooperative probing: the wave splits into groups of kProbeLanes lanes; each group
// probes one key, its lanes reading consecutive slots of the key's probe sequence at once and
// voting (ballot) for a match or a free slot.  Keys are never deleted during a call, so a key
// is absent when a free slot comes before any match.  A wave probes 64 / kProbeLanes keys at
// a time.  Returns the slot holding `key` or -1, with *free_at = the first free slot seen.
constexpr int kProbeLanes = 8;

__device__ inline int coop_find(const u64* __restrict__ hkeys, u32 hmask, u64 key, bool active,
                                u32* free_at) {
    const int lane = lane_id();
    const int sub = lane & (kProbeLanes - 1);
    const int gshift = lane - sub;                       // first lane of this group
    const u64 gmask = ((1ull << kProbeLanes) - 1ull) << gshift;
    const u32 start = (u32)mix64(key) & hmask;
    int result = -1;
    *free_at = 0xFFFFFFFFu;
    bool done = !active;
    for (u32 base = 0; base <= hmask; base += kProbeLanes) {
        if (__ballot(!done) == 0ull) break;
        const u32 slot = (start + base + (u32)sub) & hmask;
        const u64 k = done ? kEmpty : hkeys[slot];
        const u64 match = (__ballot(!done && k == key) & gmask) >> gshift;
        const u64 empty = (__ballot(!done && k == kEmpty) & gmask) >> gshift;
        if (!done) {
            const int fm = match ? __ffsll((long long)match) : 65;
            const int fe = empty ? __ffsll((long long)empty) : 65;
            if (fm < fe) {
                result = (int)((start + base + (u32)fm - 1u) & hmask);
                done = true;
            } else if (fe < 65) {
                *free_at = (start + base + (u32)fe - 1u) & hmask;
                done = true;
            }
        }
    }
    return result;
}

__global__ __launch_bounds__(256) void k_resolve(const MapDesc* __restrict__ maps,
                                                 const u64* __restrict__ tkeys,
                                                 u32* __restrict__ tval,
                                                 const u32* __restrict__ tlist,
                                                 u64* __restrict__ t_key, int* __restrict__ t_slot,
                                                 CallState* __restrict__ cs) {
    const u32 nt = cs->error ? 0u : cs->t_count;
    const int lane = lane_id();
    constexpr u32 per = 64 / kProbeLanes;          // entries per wave per round
    const u32 wave = (blockIdx.x * 256u + threadIdx.x) >> 6;
    const u32 nwaves = gridDim.x * 4u;
    for (u32 wb = wave * per; wb < nt; wb += nwaves * per) {
        // lane group g of the wave owns entry wb + g
        const u32 i = wb + (u32)lane / kProbeLanes;
        const bool act = i < nt;
        u64 key = kEmpty;
        u32 h = 0;
        if (act) {
            h = tlist[i];
            key = tkeys[h];
        }
        const MapDesc& M = maps[act ? (u32)(key >> 45) : 0u];
        u32 free_at;
        const int pos = coop_find(M.hkeys, M.hmask, key & ((1ull << 45) - 1), act, &free_at);
        if (act && (lane & (kProbeLanes - 1)) == 0) {
            tval[h] = i;
            t_key[i] = key;
            if (pos >= 0) {
                t_slot[i] = M.hslots[pos];
            } else {
                const u32 rank = atomicAdd(&M.st->new_count, 1u);
                t_slot[i] = -(int)rank - 2;   // pending: -2 - rank
            }
        }
    }
}

__global__ __launch_bounds__(256) void k_commit(const MapDesc* __restrict__ maps,
                                                const u64* __restrict__ t_key,
                                                int* __restrict__ t_slot,
                                                CallState* __restrict__ cs) {
    const u32 nt = cs->error ? 0u : cs->t_count;
    const int lane = lane_id();
    constexpr u32 per = 64 / kProbeLanes;
    const u32 wave = (blockIdx.x * 256u + threadIdx.x) >> 6;
    const u32 nwaves = gridDim.x * 4u;
    for (u32 wb = wave * per; wb < nt; wb += nwaves * per) {
        const u32 i = wb + (u32)lane / kProbeLanes;
        bool pending = false;
        u64 key = kEmpty;
        int slot = 0;
        if (i < nt) {
            key = t_key[i];
            const int sv = t_slot[i];
            if (sv <= -2) {
                const MapDesc& M = maps[(u32)(key >> 45)];
                MapState* st = M.st;
                const u32 rank = (u32)(-sv - 2);
                if (st->error == 0 && (u64)st->block_count + st->new_count <= M.capacity) {
                    pending = true;
                    slot = (int)(st->block_count + rank);
                } else {
                    st->error = -3;   // VBX_ERR_POOL_FULL: this call leaves the map unchanged
                }
            }
        }
        const MapDesc& M = maps[pending ? (u32)(key >> 45) : 0u];
        const u64 bk = key & ((1ull << 45) - 1);
        bool todo = pending;
        while (__ballot(todo) != 0ull) {
            u32 free_at;
            const int pos = coop_find(M.hkeys, M.hmask, bk, todo, &free_at);
            if (todo && (pos >= 0 || free_at == 0xFFFFFFFFu)) todo = false;   // present or full
            bool won = false;
            if (todo && (lane & (kProbeLanes - 1)) == 0) {
                won = atomicCAS(&M.hkeys[free_at], kEmpty, bk) == kEmpty;
                if (won) M.hslots[free_at] = slot;
            }
            // the group leader's outcome decides for the whole group
            const u64 wonmask = __ballot(won);
            if (todo && ((wonmask >> (lane & ~(kProbeLanes - 1))) & 1ull)) todo = false;
        }
        if (pending && (lane & (kProbeLanes - 1)) == 0) t_slot[i] = slot | (int)0x40000000;   // bit 30: new
    }
}

// ---------------------------------------------------------------------------
// bins: counting sort of crossings by (block, frame).  Projection mapping counts its crossings
// here; raycasting counts them in the crossing kernel (by block-set slot, gathered by the scan).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_bin_count(const Job* __restrict__ jobs,
                                                   const u32* __restrict__ cross,
                                                   const unsigned char* __restrict__ ncross, u32 MB,
                                                   const u32* __restrict__ tval,
                                                   const u32* __restrict__ rays_job,
                                                   u32* __restrict__ bins, u32 JM,
                                                   CallState* __restrict__ cs, u32 ray_cap) {
    const u32 nr = cs->error ? 0u : (cs->ray_count < ray_cap ? cs->ray_count : ray_cap);
    for (u32 base = blockIdx.x * 256u; base < nr; base += gridDim.x * 256u) {
        const u32 i = base + threadIdx.x;
        u32 nc = 0, jm = 0;
        if (i < nr) {
            nc = ncross[i];
            if (nc) jm = jobs[rays_job[i]].jm;
        }
        for (u32 c = 0; c < MB; ++c) {
            if (__ballot(c < nc) == 0ull) break;
            const bool act = c < nc;
            const u32 b = act ? tval[cross[(size_t)i * MB + c]] * JM + jm : 0u;
            wave_count_by_key(bins, act, b);
        }
    }
}

// Exclusive scan of bins[0, n) with n = t_count * JM, in chunks of 4096 (16 per thread).
constexpr int kScanChunk = 4096;

// Sums of the scan chunks.  The grid is sized for the largest possible count; only the
// workgroups of chunks that hold bins take part.  The last of them to finish (counted in
// cs->scan_done, which it then clears for the next scan) turns the sums into exclusive chunk
// offsets and writes the total at off[n]: no workgroup waits for another.
//
// hsrc (raycasting calls): the counts were made by block-set slot, hsrc[h * JM + frame]; they
// are moved to bins[t * JM + frame] for the dense block order t (h = tlist[t]) and cleared, so
// that hsrc is zero again for the next call, whatever the state of this one.
__global__ __launch_bounds__(256) void k_scan_sums(u32* __restrict__ bins, u32 JM,
                                                   u32* __restrict__ partial, u32* __restrict__ off,
                                                   CallState* __restrict__ cs, u32* __restrict__ hsrc,
                                                   const u32* __restrict__ tlist, u32 tlist_cap) {
    __shared__ u32 lds8[4];
    __shared__ bool s_last;
    if (hsrc) {
        const u32 tc = cs->t_count < tlist_cap ? cs->t_count : tlist_cap;   // listed blocks
        const u32 ng = tc * JM;
        const u32 gb = blockIdx.x * (u32)kScanChunk;
        for (int j = 0; j < 16; ++j) {
            const u32 i = gb + threadIdx.x * 16u + j;
            if (i < ng) {
                const u32 t = i / JM;
                const size_t src = (size_t)tlist[t] * JM + (i - t * JM);
                const u32 c = hsrc[src];
                if (c) hsrc[src] = 0u;
                bins[i] = c;
            }
        }
    }
    const u32 n = cs->error ? 0u : cs->t_count * JM;
    const u32 nparts = gridDim.x;
    const u32 used_all = (n + kScanChunk - 1) / kScanChunk;
    const u32 used = used_all < nparts ? used_all : nparts;
    if (blockIdx.x >= used) {   // whole workgroup
        if (used == 0 && blockIdx.x == 0 && threadIdx.x == 0) off[n] = 0;
        return;
    }
    const u32 base = blockIdx.x * (u32)kScanChunk;
    u32 s = 0;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        const u32 i = base + threadIdx.x * 16u + j;
        if (i < n) s += bins[i];
    }
    u32 tot;
    block_scan_256(s, lds8, &tot);
    if (threadIdx.x == 0) {
        partial[blockIdx.x] = tot;
        __threadfence();   // the sum is visible device-wide before the count says so
        s_last = atomicAdd(&cs->scan_done, 1u) == used - 1;
    }
    __syncthreads();
    if (!s_last) return;   // whole workgroup
    __threadfence();       // every other workgroup's sum is visible from here on
    if (threadIdx.x == 0) cs->scan_done = 0;
    u32 carry = 0;
    for (u32 b = 0; b < used && b < nparts; b += 256) {
        const u32 i = b + threadIdx.x;
        const u32 x = (i < used && i < nparts) ? partial[i] : 0u;
        u32 tot;
        const u32 incl = block_scan_256(x, lds8, &tot);
        if (i < used && i < nparts) partial[i] = carry + incl - x;
        carry += tot;
    }
    if (threadIdx.x == 0) off[n] = carry;
}

// With chunk_first (the partial-group sort), it also records the first bin of every merge chunk:
// chunk_first[c] = the first bin whose first partial lies at or after c * kMergeSpan, i.e. bin
// b for the chunks whose start lies in (off[b - 1], off[b]], and the end n for those up to off[n].
__global__ __launch_bounds__(256) void k_scan_final(const u32* __restrict__ bins,
                                                    const u32* __restrict__ partial,
                                                    u32* __restrict__ off, u32 JM,
                                                    u32* __restrict__ chunk_first,
                                                    const CallState* __restrict__ cs) {
    __shared__ u32 lds8[4];
    const u32 n = cs->error ? 0u : cs->t_count * JM;
    const u32 base = blockIdx.x * (u32)kScanChunk;
    if (base >= n) return;
    u32 v[16];
    u32 s = 0;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        const u32 i = base + threadIdx.x * 16u + j;
        v[j] = i < n ? bins[i] : 0u;
        s += v[j];
    }
    u32 tot;
    const u32 incl = block_scan_256(s, lds8, &tot);
    u32 run = partial[blockIdx.x] + incl - s;
    const u32 i0 = base + threadIdx.x * 16u;
    u32 prev = chunk_first && i0 > 0u && i0 < n ? run - bins[i0 - 1u] : 0u;   // off[i - 1]
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        const u32 i = i0 + j;
        if (i < n) {
            off[i] = run;
            if (chunk_first) {
                for (u32 c = i == 0u ? 0u : prev / kMergeSpan + 1u; c <= run / kMergeSpan; ++c)
                    chunk_first[c] = i;
                prev = run;
                if (i + 1u == n)
                    for (u32 c = prev / kMergeSpan + 1u; c <= (run + v[j]) / kMergeSpan; ++c)
                        chunk_first[c] = n;
            }
        }
        run += v[j];
    }
}

// Copies each crossing's ray (end point, weight) to its bin position, so that the update
// kernel reads every (block, frame) bin contiguously.  Counts are decremented back to zero,
// leaving the bins clean for the next call.
__global__ __launch_bounds__(256) void k_scatter(const Job* __restrict__ jobs,
                                                 const u32* __restrict__ cross,
                                                 const unsigned char* __restrict__ ncross, u32 MB,
                                                 const u32* __restrict__ tval,
                                                 const u32* __restrict__ rays_job,
                                                 u32* __restrict__ bins, const u32* __restrict__ off,
                                                 u32 JM, const float4* __restrict__ rays_p,
                                                 float4* __restrict__ sorted,
                                                 const u32* __restrict__ rays_c, u32* __restrict__ sorted_c,
                                                 CallState* __restrict__ cs, u32 ray_cap) {
    const u32 nr = cs->error ? 0u : (cs->ray_count < ray_cap ? cs->ray_count : ray_cap);
    for (u32 base = blockIdx.x * 256u; base < nr; base += gridDim.x * 256u) {
        const u32 i = base + threadIdx.x;
        u32 nc = 0, jm = 0;
        float4 rp = make_float4(0.f, 0.f, 0.f, 0.f);
        u32 col = 0;
        if (i < nr) {
            nc = ncross[i];
            if (nc) {
                jm = jobs[rays_job[i]].jm;
                rp = rays_p[i];
                if (rays_c) col = rays_c[i];
            }
        }
        for (u32 c = 0; c < MB; ++c) {
            if (__ballot(c < nc) == 0ull) break;
            const bool act = c < nc;
            const u32 b = act ? tval[cross[(size_t)i * MB + c]] * JM + jm : 0u;
            // lanes sharing a bin take consecutive positions reserved by one atomic
            const u32 pos = wave_claim_by_key(bins, off, act, b);
            if (act) sorted[pos] = rp;
            if (act && sorted_c) sorted_c[pos] = col;
        }
    }
}

// ---------------------------------------------------------------------------
// update: one workgroup per touched block
// ---------------------------------------------------------------------------
template <int STORAGE>
__device__ inline void store_voxel(void* pool, size_t idx, float D, float W) {
    if (STORAGE == 0) {
        ((float2*)pool)[idx] = make_float2(D, W);
    } else {
        const u32 d = STORAGE == 1 ? (u32)__half_as_ushort(__float2half_rn(D)) : (u32)s16_encode(D);
        const u32 w = __half_as_ushort(__float2half_rn(W));
        ((u32*)pool)[idx] = d | (w << 16);
    }
}

// The stored value a binary32 result of Eqs. (3)-(4) becomes (rounded once per frame).
template <int STORAGE>
__device__ inline void round_to_storage(float& D, float& W) {
    if (STORAGE == 1) {
        D = __half2float(__float2half_rn(D));
        W = __half2float(__float2half_rn(W));
    } else if (STORAGE == 2) {
        D = s16_decode(s16_encode(D));
        W = __half2float(__float2half_rn(W));
    }
}

// A fixed-point sum (below 2^62 in magnitude) to binary32: its two 32-bit halves convert to
// binary64 exactly and one fma joins them (exact below 2^53, else rounded once), then one
// rounding to binary32 -- within 2^-24 + 2^-53 of the sum relative to it, in a few
// instructions instead of the integer normalisation of a direct 64-bit conversion.
__device__ inline float fixed_to_float(u64 x) {
    return (float)__builtin_fma((double)(u32)(x >> 32), 0x1p32, (double)(u32)x);
}
__device__ inline float fixed_to_float(i64 x) {
    return (float)__builtin_fma((double)(int)(x >> 32), 0x1p32, (double)(u32)(u64)x);
}

constexpr int kOffWindow = 256;   // frames whose bin offsets are staged in LDS at a time

// Order in which the update takes the call's blocks: heaviest first (log2 buckets of the rays
// crossing the block over all frames of the call), so that the longest frame chains start at
// once and the light blocks fill in behind them.  One workgroup; the order within a bucket is
// free (each block is folded by one workgroup, so results do not depend on it).
__global__ __launch_bounds__(1024) void k_order_blocks(const u32* __restrict__ off, u32 JM,
                                                       u32* __restrict__ order,
                                                       const CallState* __restrict__ cs) {
    __shared__ u32 s_cnt[33];
    __shared__ u32 s_base[33];
    const u32 nt = cs->error ? 0u : cs->t_count;
    if (threadIdx.x < 33) s_cnt[threadIdx.x] = 0;
    __syncthreads();
    for (u32 t = threadIdx.x; t < nt; t += 1024) {
        const u32 w = off[(t + 1) * JM] - off[t * JM];
        atomicAdd(&s_cnt[w ? 32 - __clz(w) : 0], 1u);   // bucket: bit length of w
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        u32 acc = 0;
        for (int b = 32; b >= 0; --b) { s_base[b] = acc; acc += s_cnt[b]; }   // heaviest first
    }
    __syncthreads();
    for (u32 t = threadIdx.x; t < nt; t += 1024) {
        const u32 w = off[(t + 1) * JM] - off[t * JM];
        order[atomicAdd(&s_base[w ? 32 - __clz(w) : 0], 1u)] = t;
    }
}

// Work item u = t * NREG + q: region q of touched block t, a box of RX x RY x RZ voxels
// (regions tile the block, x fastest).  Regions of one block are independent (different
// voxels) and replay the same rays, each ray walked in full but observed only inside the
// region, so a block's frames run in parallel across NREG workgroups with 1/NREG of the LDS
// each.  z-slabs divide the rays of walls, x/y columns those of floors and walls alike.
//
// COLOR (maps that keep colour, one frame per step): each voxel also sums weight * channel of
// the frame's rays (scale 2^(kw - 8)) and, before Eq. (4) changes W, folds the frame's mean ray
// colour into its colour with the weight from before the frame (Sec. IV-B):
//   C <- round((W C + sum w c) / (W + sum w)),  binary64 quotient, rounded to even.
template <int STORAGE, int RX, int RY, int RZ, int NT, bool COLOR>
__global__ __launch_bounds__(NT) void k_update(const Job* __restrict__ jobs,
                                                const MapDesc* __restrict__ maps,
                                                const u64* __restrict__ t_key,
                                                const int* __restrict__ t_slot,
                                                const u32* __restrict__ off,
                                                const u32* __restrict__ order,
                                                const float4* __restrict__ sorted,
                                                const u32* __restrict__ sorted_c, u32 JM,
                                                u64* __restrict__ touch_key,
                                                u32* __restrict__ touch_n, u32 touch_cap,
                                                int keep_touches,
                                                JobStat* __restrict__ jst,
                                                CallState* __restrict__ cs) {
    constexpr int VOX = RX * RY * RZ;      // voxels of one region
    constexpr int VPT = VOX / NT;          // voxels per thread
    constexpr int NRX = 16 / RX, NRY = 16 / RY, NRZ = 16 / RZ;
    constexpr int NREG = NRX * NRY * NRZ;  // regions per block
    static_assert(VPT * NT == VOX && VPT >= 1, "region size must be a multiple of the workgroup");
    // With 1024-thread workgroups (which the thread limit already keeps to two per CU, so the
    // second set of sums costs no occupancy) frames are taken two at a time: each half of the
    // workgroup walks one frame into its own sums, then every voxel folds the earlier frame and
    // then the later one.  A voxel's ray count over the call (a_c) grows by 1 per ray of the
    // earlier frame and by 2^16 per ray of the later one, which splits exactly while each frame
    // has fewer than 2^16 rays in the block; a frame with more is walked alone.  Smaller
    // workgroups walk one frame at a time.
    constexpr int K = NT == 1024 ? 2 : 1;
    static_assert(!COLOR || K == 1, "colour sums are kept for one frame per step");
    __shared__ u64 a_sc[3][COLOR ? VOX : 1];   // colour maps: weight * channel sums of the frame
    __shared__ u64 a_w[K][VOX];   // sum of fixed-point weights, per frame of the step
    __shared__ u64 a_d[K][VOX];   // sum of fixed-point weight * distance/delta (two's complement)
    __shared__ u32 a_c[VOX];      // rays over the call (see above)
    __shared__ u32 s_off[kOffWindow + 1];
    __shared__ unsigned short s_fr[kOffWindow];   // the window's frames with rays, in order
    __shared__ u32 s_wcnt[kOffWindow / 64];       // their count per wave of the listing
    __shared__ u32 s_t;
    __shared__ u32 s_stat[3];
    __shared__ u32 s_tbase;
    __shared__ u32 lds8[NT / 64];
    static_assert(NT % (64 * K) == 0, "each half of the workgroup is whole waves");
    static_assert(NT >= kOffWindow, "one thread per frame of a window");
    // Lists the frames of the staged window (wn of them) that have rays in s_fr, in order;
    // returns their count (the same in every thread).  Called by every thread.
    auto list_frames = [&](int wn) -> int {
        const int j = (int)threadIdx.x, wave = j >> 6, lane = lane_id();
        const bool has = j < wn && s_off[j + 1] > s_off[j];
        const u64 bal = __ballot(has);
        if (wave < kOffWindow / 64 && lane == 0) s_wcnt[wave] = (u32)__popcll(bal);
        __syncthreads();
        u32 base = 0, tot = 0;
#pragma unroll
        for (int v = 0; v < kOffWindow / 64; ++v) {
            base += v < wave ? s_wcnt[v] : 0u;
            tot += s_wcnt[v];
        }
        if (has) s_fr[base + (u32)__popcll(bal & ((1ull << lane) - 1ull))] = (unsigned short)j;
        __syncthreads();
        return __builtin_amdgcn_readfirstlane((int)tot);
    };
    for (int i = threadIdx.x; i < VOX; i += NT) {
        a_c[i] = 0;
#pragma unroll
        for (int h = 0; h < K; ++h) { a_w[h][i] = 0; a_d[h][i] = 0; }
        if (COLOR) { a_sc[0][i] = 0; a_sc[1][i] = 0; a_sc[2][i] = 0; }
    }
    const u32 nt = cs->error ? 0u : cs->t_count * (u32)NREG;
    for (;;) {
        if (threadIdx.x == 0) { s_t = atomicAdd(&cs->work_next, 1u); s_stat[0] = 0; s_stat[1] = 0; s_stat[2] = 0; }
        __syncthreads();
        const u32 u = s_t;
        if (u >= nt) break;
        const u32 t = order[u / (u32)NREG];    // heaviest blocks first
        const int q = (int)(u % (u32)NREG);
        const int qx = q % NRX, qy = (q / NRX) % NRY, qz = q / (NRX * NRY);
        const u64 tk = t_key[t];
        // by value: the walk loop then reads the map constants from registers instead of
        // reloading them after every LDS atomic
        const MapDesc M = maps[(u32)(tk >> 45)];
        if (M.st->error != 0) { __syncthreads(); continue; }
        int bx, by, bz;
        unpack_block(tk & ((1ull << 45) - 1), bx, by, bz);
        const int ts = t_slot[t];
        const bool is_new = (ts & 0x40000000) != 0;
        const size_t slot = (size_t)(ts & 0x3FFFFFFF);
        void* pool = M.pool;
        // voxel i of the region (i = threadIdx.x + NT * j) is block voxel pool_index(i)
        const size_t vbase = slot * 4096 + (size_t)(qx * RX + 16 * (qy * RY) + 256 * (qz * RZ));
        auto block_local = [](int i) { return (i % RX) + 16 * ((i / RX) % RY) + 256 * (i / (RX * RY)); };
        float D[VPT], W[VPT];
        u32 ntot[VPT], last[VPT];
        u32 C[COLOR ? VPT : 1];
        // a map without colour can share a colour call with maps that keep it
        const bool has_color = COLOR && M.color != nullptr;
#pragma unroll
        for (int j = 0; j < VPT; ++j) {
            ntot[j] = 0;
            if (COLOR) C[j] = (is_new || !has_color) ? 0u : M.color[vbase + block_local(threadIdx.x + NT * j)];
            if constexpr (K == 2) {   // one frame at a time leaves the counts cleared by its folds
                last[j] = 0;
                a_c[threadIdx.x + NT * j] = 0;
            }
            if (is_new) { D[j] = 0.0f; W[j] = 0.0f; }
            else load_voxel<STORAGE>(pool, vbase + block_local(threadIdx.x + NT * j), D[j], W[j]);
        }
        const int ox = 16 * bx + qx * RX, oy = 16 * by + qy * RY, oz = 16 * bz + qz * RZ;
        u32 stat_vox = 0, stat_touch = 0;
        if constexpr (K == 2) {
            for (int w0 = 0; w0 < M.njobs; w0 += kOffWindow) {
                const int wn = M.njobs - w0 < kOffWindow ? M.njobs - w0 : kOffWindow;
                for (int k = threadIdx.x; k <= wn; k += NT) s_off[k] = off[t * JM + (u32)(w0 + k)];
                __syncthreads();
                const int nfr = list_frames(wn);
                // Step plan from the window's offsets (the same in every thread): the step's first
                // frame jm (the im-th frame with rays), the next frame with rays jn, whether the two
                // are walked together, and this thread's frame, position and stride in that frame's
                // rays.
                auto fr_at = [&](int i) { return i < nfr ? __builtin_amdgcn_readfirstlane((int)s_fr[i]) : wn; };
                struct Step {
                    int im, jm, jn, fr;
                    bool pair;
                    u32 pos, stride, cadd;
                    int half;
                };
                auto plan = [&](int im) {
                    Step S;
                    S.im = im;
                    S.jm = fr_at(im);
                    S.jn = S.jm < wn ? fr_at(im + 1) : wn;
                    S.pair = K == 2 && S.jn < wn && s_off[S.jm + 1] - s_off[S.jm] < 65536u &&
                             s_off[S.jn + 1] - s_off[S.jn] < 65536u;
                    S.half = S.pair && (int)threadIdx.x >= NT / 2 ? 1 : 0;
                    S.fr = S.half ? S.jn : S.jm;
                    S.pos = S.half ? threadIdx.x - NT / 2 : threadIdx.x;
                    S.stride = S.pair ? NT / 2 : NT;
                    S.cadd = S.half ? 65536u : 1u;
                    return S;
                };
                // the first ray and sensor origin of every thread for the next step are loaded while
                // the current step is processed
                Step S = plan(0);
                float4 nxt = make_float4(0.f, 0.f, 0.f, 0.f);
                float nxs[3] = {0.f, 0.f, 0.f};
                if (S.jm < wn) {
                    const u32 e = s_off[S.fr] + S.pos;
                    if (e < s_off[S.fr + 1]) nxt = sorted[e];
                    const Job& Jn = jobs[M.job0 + w0 + S.fr];
                    nxs[0] = Jn.pose[3]; nxs[1] = Jn.pose[7]; nxs[2] = Jn.pose[11];
                }
                while (S.jm < wn) {
                    const Step Sn = plan(S.pair ? S.im + 2 : S.im + 1);
                    const float4 cur = nxt;
                    const float s[3] = {nxs[0], nxs[1], nxs[2]};
                    const u32 lo = s_off[S.fr], hi = s_off[S.fr + 1];
                    if (Sn.jm < wn) {
                        const u32 e = s_off[Sn.fr] + Sn.pos;
                        if (e < s_off[Sn.fr + 1]) nxt = sorted[e];
                        const Job& Jn = jobs[M.job0 + w0 + Sn.fr];
                        nxs[0] = Jn.pose[3]; nxs[1] = Jn.pose[7]; nxs[2] = Jn.pose[11];
                    }
                    u64* const sw_buf = a_w[K == 2 ? S.half : 0];
                    u64* const sd_buf = a_d[K == 2 ? S.half : 0];
                    float4 rp = cur;
                    for (u32 e = lo + S.pos; e < hi; e += S.stride) {
                        // the next ray's load is in flight while this one is walked
                        float4 rn = make_float4(0.f, 0.f, 0.f, 0.f);
                        if (e + S.stride < hi) rn = sorted[e + S.stride];
                        const float p[3] = {rp.x, rp.y, rp.z};
                        // the ray weight in fixed-point units: scaling by the power of two 2^kw
                        // here rather than after the products leaves every product unchanged
                        const float wgt = rp.w * M.wscale;
                        rp = rn;
                        float ev[3], r;
                        Walk w;
                        walk_setup(M, p, s, ev, r, w);
                        if (NREG > 1) {
                            // every walk index lies between its end voxels: skip bands that miss the region
                            const int o3[3] = {ox, oy, oz};
                            const int r3[3] = {RX, RY, RZ};
                            bool miss = false;
    #pragma unroll
                            for (int a = 0; a < 3; ++a) {
                                const int g_end = w.g[a] + w.step[a] * w.n[a];
                                const int glo = w.g[a] < g_end ? w.g[a] : g_end;
                                const int ghi = w.g[a] < g_end ? g_end : w.g[a];
                                miss = miss || ghi < o3[a] || glo >= o3[a] + r3[a];
                            }
                            if (miss) continue;
                        }
                        // the walk through the region, with the distance form fixed per ray
                        auto walk_band = [&](auto dist_form) {
                            constexpr int DIST = decltype(dist_form)::value;
                            bool inside = false;
                            for (int guard = 0; guard < M.max_steps; ++guard) {
                                const int lx = w.g[0] - ox, ly = w.g[1] - oy, lz = w.g[2] - oz;
                                // (bitwise operators: no branch per test)
                                const bool in = ((u32)lx < (u32)RX) & ((u32)ly < (u32)RY) & ((u32)lz < (u32)RZ);
                                if (in) {
                                    const Obs o = observe<DIST>(M, p, ev, r, wgt, w.g[0], w.g[1], w.g[2]);
                                    const u32 l = (u32)lx + (u32)RX * ((u32)ly + (u32)RY * (u32)lz);
                                    u64 fw, fd;
                                    fixed_terms(o.w, o.w * o.e, fw, fd);
                                    // issued unconditionally: a wave issues an LDS atomic once for
                                    // all its lanes, and adding zero is harmless
                                    atomicAdd(&sw_buf[l], fw);
                                    atomicAdd(&sd_buf[l], fd);
                                    atomicAdd(&a_c[l], S.cadd);
                                }
                                // one exit: the walk's last voxel, or the first voxel after the region
                                // (the walk is monotone per axis: it never re-enters the region)
                                const bool stop = (inside & !in) | (w.left == 0);
                                inside |= in;
                                if (stop) break;
                                walk_step(w);
                            }
                        };
                        if (M.dist == 0) walk_band(std::integral_constant<int, 0>{});
                        else walk_band(std::integral_constant<int, 1>{});
                    }
                    __syncthreads();
                    // Eqs. (3)-(4), once per voxel for each frame of the step, in frame order.
                    // (The counts of all this thread's voxels are read together, and each sum
                    // pair together: LDS reads in flight at once rather than one after another.)
                    u32 cnt_all[VPT];
    #pragma unroll
                    for (int j = 0; j < VPT; ++j) cnt_all[j] = a_c[threadIdx.x + NT * j];
    #pragma unroll
                    for (int j = 0; j < VPT; ++j) {
                        const int l = threadIdx.x + NT * j;
                        const u32 c = cnt_all[j];
                        const u32 d = c - last[j];
                        last[j] = c;
                        const u32 dn[2] = {S.pair ? (d & 0xFFFFu) : d, S.pair ? (d >> 16) : 0u};
    #pragma unroll
                        for (int h = 0; h < K; ++h) {
                            if (!dn[h]) continue;
                            const u64 sw_fx = a_w[h][l], sd_fx = a_d[h][l];
                            if (sw_fx) {
                                const float sw = fixed_to_float(sw_fx) * M.inv_wscale;
                                // sums are in units of delta; binary32 storage keeps D in metres,
                                // 16-bit storage keeps D / delta
                                float swd = fixed_to_float((i64)sd_fx) * M.inv_wscale;
                                if (STORAGE == 0) swd = swd * M.delta;
                                float Dn = (W[j] * D[j] + swd) / (W[j] + sw);
                                float Wn = W[j] + sw;
                                if (Wn > M.w_max) Wn = M.w_max;
                                round_to_storage<STORAGE>(Dn, Wn);
                                D[j] = Dn;
                                W[j] = Wn;
                            }
                            ntot[j] += dn[h];
                            stat_vox += 1;
                            stat_touch += dn[h];
                            a_w[h][l] = 0; a_d[h][l] = 0;
                        }
                    }
                    __syncthreads();
                    S = Sn;
                }
                __syncthreads();
            }
        } else {
            // one frame at a time: a_c holds the frame's ray counts, cleared by the fold
            for (int w0 = 0; w0 < M.njobs; w0 += kOffWindow) {
                const int wn = M.njobs - w0 < kOffWindow ? M.njobs - w0 : kOffWindow;
                for (int k = threadIdx.x; k <= wn; k += NT) s_off[k] = off[t * JM + (u32)(w0 + k)];
                __syncthreads();
                const int nfr = list_frames(wn);
                // frames of the window with rays in order (the im-th is jm); the first ray of every
                // thread for the next one is loaded while the current frame is processed
                int im = 0;
                int jm = nfr > 0 ? __builtin_amdgcn_readfirstlane((int)s_fr[0]) : wn;
                float4 nxt = make_float4(0.f, 0.f, 0.f, 0.f);
                u32 nxc = 0;                       // colour maps: the ray's colour, loaded with it
                float nxs[3] = {0.f, 0.f, 0.f};   // that frame's sensor origin, also loaded ahead
                if (jm < wn) {
                    const u32 e = s_off[jm] + threadIdx.x;
                    if (e < s_off[jm + 1]) { nxt = sorted[e]; if (COLOR) nxc = sorted_c[e]; }
                    const Job& Jn = jobs[M.job0 + w0 + jm];
                    nxs[0] = Jn.pose[3]; nxs[1] = Jn.pose[7]; nxs[2] = Jn.pose[11];
                }
                while (jm < wn) {
                    const int jn = im + 1 < nfr ? __builtin_amdgcn_readfirstlane((int)s_fr[im + 1]) : wn;
                    const float4 cur = nxt;
                    const u32 curc = nxc;
                    const float s[3] = {nxs[0], nxs[1], nxs[2]};
                    const u32 lo = s_off[jm], hi = s_off[jm + 1];
                    if (jn < wn) {
                        const u32 e = s_off[jn] + threadIdx.x;
                        if (e < s_off[jn + 1]) { nxt = sorted[e]; if (COLOR) nxc = sorted_c[e]; }
                        const Job& Jn = jobs[M.job0 + w0 + jn];
                        nxs[0] = Jn.pose[3]; nxs[1] = Jn.pose[7]; nxs[2] = Jn.pose[11];
                    }
                    float4 rp = cur;
                    u32 rc = curc;
                    for (u32 e = lo + threadIdx.x; e < hi; e += NT) {
                        // the next ray's load is in flight while this one is walked
                        float4 rn = make_float4(0.f, 0.f, 0.f, 0.f);
                        u32 rnc = 0;
                        if (e + NT < hi) { rn = sorted[e + NT]; if (COLOR) rnc = sorted_c[e + NT]; }
                        const float p[3] = {rp.x, rp.y, rp.z};
                        // the ray weight in fixed-point units: scaling by the power of two 2^kw
                        // here rather than after the products leaves every product unchanged
                        const float wgt = rp.w * M.wscale;
                        const float cf[3] = {(float)(rc & 255u), (float)((rc >> 8) & 255u), (float)((rc >> 16) & 255u)};
                        rp = rn;
                        rc = rnc;
                        float ev[3], r;
                        Walk w;
                        walk_setup(M, p, s, ev, r, w);
                        if (NREG > 1) {
                            // every walk index lies between its end voxels: skip bands that miss the region
                            const int o3[3] = {ox, oy, oz};
                            const int r3[3] = {RX, RY, RZ};
                            bool miss = false;
    #pragma unroll
                            for (int a = 0; a < 3; ++a) {
                                const int g_end = w.g[a] + w.step[a] * w.n[a];
                                const int glo = w.g[a] < g_end ? w.g[a] : g_end;
                                const int ghi = w.g[a] < g_end ? g_end : w.g[a];
                                miss = miss || ghi < o3[a] || glo >= o3[a] + r3[a];
                            }
                            if (miss) continue;
                        }
                        // the walk through the region, with the distance form fixed per ray
                        auto walk_band = [&](auto dist_form) {
                            constexpr int DIST = decltype(dist_form)::value;
                            bool inside = false;
                            for (int guard = 0; guard < M.max_steps; ++guard) {
                                const int lx = w.g[0] - ox, ly = w.g[1] - oy, lz = w.g[2] - oz;
                                // (bitwise operators: no branch per test)
                                const bool in = ((u32)lx < (u32)RX) & ((u32)ly < (u32)RY) & ((u32)lz < (u32)RZ);
                                if (in) {
                                    const Obs o = observe<DIST>(M, p, ev, r, wgt, w.g[0], w.g[1], w.g[2]);
                                    const u32 l = (u32)lx + (u32)RX * ((u32)ly + (u32)RY * (u32)lz);
                                    u64 fw, fd;
                                    fixed_terms(o.w, o.w * o.e, fw, fd);
                                    // issued unconditionally: a wave issues an LDS atomic once for
                                    // all its lanes, and adding zero is harmless
                                    atomicAdd(&a_w[0][l], fw);
                                    atomicAdd(&a_d[0][l], fd);
                                    atomicAdd(&a_c[l], 1u);
                                    if (COLOR) {
                                        const float cscale = 1.0f / 256.0f;   // o.w carries 2^kw
    #pragma unroll
                                        for (int k = 0; k < 3; ++k)
                                            atomicAdd(&a_sc[k][l], (u64)__builtin_rintf(o.w * cf[k] * cscale));
                                    }
                                }
                                // one exit: the walk's last voxel, or the first voxel after the region
                                // (the walk is monotone per axis: it never re-enters the region)
                                const bool stop = (inside & !in) | (w.left == 0);
                                inside |= in;
                                if (stop) break;
                                walk_step(w);
                            }
                        };
                        if (M.dist == 0) walk_band(std::integral_constant<int, 0>{});
                        else walk_band(std::integral_constant<int, 1>{});
                    }
                    __syncthreads();
                    // Eqs. (3)-(4), once per voxel for this frame (counts read together, and
                    // each sum pair together, as above)
                    u32 cnt_all[VPT];
    #pragma unroll
                    for (int j = 0; j < VPT; ++j) cnt_all[j] = a_c[threadIdx.x + NT * j];
    #pragma unroll
                    for (int j = 0; j < VPT; ++j) {
                        const int l = threadIdx.x + NT * j;
                        const u32 c = cnt_all[j];
                        if (c) {
                            const u64 sw_fx = a_w[0][l], sd_fx = a_d[0][l];
                            if (has_color && sw_fx) {
                                // colour first, with the weight from before the frame
                                const double swd64 = (double)sw_fx * (double)M.inv_wscale, Wd = (double)W[j];
                                const double inv_c = (double)M.inv_wscale * 256.0;
                                u32 cn = 0;
#pragma unroll
                                for (int k = 0; k < 3; ++k) {
                                    const double ck = (double)((C[j] >> (8 * k)) & 255u);
                                    double q = __builtin_rint((Wd * ck + (double)a_sc[k][l] * inv_c) / (Wd + swd64));
                                    q = q < 0.0 ? 0.0 : (q > 255.0 ? 255.0 : q);
                                    cn |= (u32)q << (8 * k);
                                }
                                C[j] = cn;
                            }
                            if (COLOR) { a_sc[0][l] = 0; a_sc[1][l] = 0; a_sc[2][l] = 0; }
                            if (sw_fx) {
                                const float sw = fixed_to_float(sw_fx) * M.inv_wscale;
                                // sums are in units of delta; binary32 storage keeps D in metres,
                                // 16-bit storage keeps D / delta
                                float swd = fixed_to_float((i64)sd_fx) * M.inv_wscale;
                                if (STORAGE == 0) swd = swd * M.delta;
                                float Dn = (W[j] * D[j] + swd) / (W[j] + sw);
                                float Wn = W[j] + sw;
                                if (Wn > M.w_max) Wn = M.w_max;
                                round_to_storage<STORAGE>(Dn, Wn);
                                D[j] = Dn;
                                W[j] = Wn;
                            }
                            ntot[j] += c;
                            stat_vox += 1;
                            stat_touch += c;
                            a_w[0][l] = 0; a_d[0][l] = 0; a_c[l] = 0;
                        }
                    }
                    __syncthreads();
                    jm = jn;
                    ++im;
                }
                __syncthreads();
            }
        }
#pragma unroll
        for (int j = 0; j < VPT; ++j) store_voxel<STORAGE>(pool, vbase + block_local(threadIdx.x + NT * j), D[j], W[j]);
        if (has_color)
#pragma unroll
            for (int j = 0; j < VPT; ++j) M.color[vbase + block_local(threadIdx.x + NT * j)] = C[j];
        if (threadIdx.x == 0 && M.dirty) M.dirty[slot] = 1u;   // the ESDF layer looks at this block again
        {
            // summed over the wave first: one lane adds (an atomic on one address with a
            // different value per lane is otherwise carried out lane by lane)
            u32 cells = 0;
#pragma unroll
            for (int j = 0; j < VPT; ++j) cells += ntot[j] ? 1u : 0u;
            const u32 wv = wave_sum(stat_vox), wt = wave_sum(stat_touch), wc = wave_sum(cells);
            if (lane_id() == 0 && wv) {
                atomicAdd(&s_stat[0], wv);
                atomicAdd(&s_stat[1], wt);
                atomicAdd(&s_stat[2], wc);
            }
        }
        if (keep_touches) {
            u32 mine = 0;
#pragma unroll
            for (int j = 0; j < VPT; ++j) mine += ntot[j] ? 1u : 0u;
            u32 tot;
            const u32 incl = block_scan<NT>(mine, lds8, &tot);
            if (threadIdx.x == 0) s_tbase = atomicAdd(&cs->touch_count, tot);
            __syncthreads();
            u32 pos = s_tbase + incl - mine;
#pragma unroll
            for (int j = 0; j < VPT; ++j) {
                if (ntot[j]) {
                    const int l = threadIdx.x + NT * j;
                    if (pos < touch_cap) {
                        touch_key[pos] = ((u64)(M.map_id) << 57) |
                                         voxel_key_of(ox + l % RX, oy + (l / RX) % RY, oz + l / (RX * RY));
                        touch_n[pos] = ntot[j];
                    }
                    pos++;
                }
            }
        }
        __syncthreads();
        if (threadIdx.x == 0 && s_stat[0]) {
            atomicAdd(&jst[M.job0].voxels, (u64)s_stat[0]);
            atomicAdd(&jst[M.job0].touches, (u64)s_stat[1]);
            atomicAdd(&jst[M.job0].cells, (u64)s_stat[2]);
        }
        __syncthreads();
    }
}

template __global__ void k_update<0, 16, 16, 16, 256, false>(const Job*, const MapDesc*, const u64*, const int*,
                                                        const u32*, const u32*, const float4*, const u32*, u32, u64*, u32*, u32,
                                                        int, JobStat*, CallState*);
template __global__ void k_update<0, 16, 16, 8, 256, false>(const Job*, const MapDesc*, const u64*, const int*,
                                                        const u32*, const u32*, const float4*, const u32*, u32, u64*, u32*, u32,
                                                        int, JobStat*, CallState*);
template __global__ void k_update<0, 16, 16, 4, 256, false>(const Job*, const MapDesc*, const u64*, const int*,
                                                        const u32*, const u32*, const float4*, const u32*, u32, u64*, u32*, u32,
                                                        int, JobStat*, CallState*);
template __global__ void k_update<0, 8, 16, 16, 256, false>(const Job*, const MapDesc*, const u64*, const int*,
                                                        const u32*, const u32*, const float4*, const u32*, u32, u64*, u32*, u32,
                                                        int, JobStat*, CallState*);
template __global__ void k_update<0, 8, 8, 16, 256, false>(const Job*, const MapDesc*, const u64*, const int*,
                                                        const u32*, const u32*, const float4*, const u32*, u32, u64*, u32*, u32,
                                                        int, JobStat*, CallState*);
template __global__ void k_update<0, 4, 8, 16, 256, false>(const Job*, const MapDesc*, const u64*, const int*,
                                                        const u32*, const u32*, const float4*, const u32*, u32, u64*, u32*, u32,
                                                        int, JobStat*, CallState*);
template __global__ void k_update<0, 16, 16, 16, 1024, false>(const Job*, const MapDesc*, const u64*, const int*,
                                                        const u32*, const u32*, const float4*, const u32*, u32, u64*, u32*, u32,
                                                        int, JobStat*, CallState*);
template __global__ void k_update<0, 16, 16, 8, 1024, false>(const Job*, const MapDesc*, const u64*, const int*,
                                                        const u32*, const u32*, const float4*, const u32*, u32, u64*, u32*, u32,
                                                        int, JobStat*, CallState*);
template __global__ void k_update<0, 16, 16, 4, 1024, false>(const Job*, const MapDesc*, const u64*, const int*,
                                                        const u32*, const u32*, const float4*, const u32*, u32, u64*, u32*, u32,
                                                        int, JobStat*, CallState*);
template __global__ void k_update<0, 16, 16, 8, 512, false>(const Job*, const MapDesc*, const u64*, const int*,
                                                        const u32*, const u32*, const float4*, const u32*, u32, u64*, u32*, u32,
                                                        int, JobStat*, CallState*);
template __global__ void k_update<1, 16, 16, 16, 256, false>(const Job*, const MapDesc*, const u64*, const int*,
                                                        const u32*, const u32*, const float4*, const u32*, u32, u64*, u32*, u32,
                                                        int, JobStat*, CallState*);
template __global__ void k_update<1, 16, 16, 8, 256, false>(const Job*, const MapDesc*, const u64*, const int*,
                                                        const u32*, const u32*, const float4*, const u32*, u32, u64*, u32*, u32,
                                                        int, JobStat*, CallState*);
template __global__ void k_update<1, 16, 16, 4, 256, false>(const Job*, const MapDesc*, const u64*, const int*,
                                                        const u32*, const u32*, const float4*, const u32*, u32, u64*, u32*, u32,
                                                        int, JobStat*, CallState*);
template __global__ void k_update<1, 8, 16, 16, 256, false>(const Job*, const MapDesc*, const u64*, const int*,
                                                        const u32*, const u32*, const float4*, const u32*, u32, u64*, u32*, u32,
                                                        int, JobStat*, CallState*);
template __global__ void k_update<1, 8, 8, 16, 256, false>(const Job*, const MapDesc*, const u64*, const int*,
                                                        const u32*, const u32*, const float4*, const u32*, u32, u64*, u32*, u32,
                                                        int, JobStat*, CallState*);
template __global__ void k_update<1, 4, 8, 16, 256, false>(const Job*, const MapDesc*, const u64*, const int*,
                                                        const u32*, const u32*, const float4*, const u32*, u32, u64*, u32*, u32,
                                                        int, JobStat*, CallState*);
template __global__ void k_update<1, 16, 16, 16, 1024, false>(const Job*, const MapDesc*, const u64*, const int*,
                                                        const u32*, const u32*, const float4*, const u32*, u32, u64*, u32*, u32,
                                                        int, JobStat*, CallState*);
template __global__ void k_update<1, 16, 16, 8, 1024, false>(const Job*, const MapDesc*, const u64*, const int*,
                                                        const u32*, const u32*, const float4*, const u32*, u32, u64*, u32*, u32,
                                                        int, JobStat*, CallState*);
template __global__ void k_update<1, 16, 16, 4, 1024, false>(const Job*, const MapDesc*, const u64*, const int*,
                                                        const u32*, const u32*, const float4*, const u32*, u32, u64*, u32*, u32,
                                                        int, JobStat*, CallState*);
template __global__ void k_update<1, 16, 16, 8, 512, false>(const Job*, const MapDesc*, const u64*, const int*,
                                                        const u32*, const u32*, const float4*, const u32*, u32, u64*, u32*, u32,
                                                        int, JobStat*, CallState*);
template __global__ void k_update<2, 16, 16, 16, 256, false>(const Job*, const MapDesc*, const u64*, const int*,
                                                        const u32*, const u32*, const float4*, const u32*, u32, u64*, u32*, u32,
                                                        int, JobStat*, CallState*);
template __global__ void k_update<2, 16, 16, 8, 256, false>(const Job*, const MapDesc*, const u64*, const int*,
                                                        const u32*, const u32*, const float4*, const u32*, u32, u64*, u32*, u32,
                                                        int, JobStat*, CallState*);
template __global__ void k_update<2, 16, 16, 4, 256, false>(const Job*, const MapDesc*, const u64*, const int*,
                                                        const u32*, const u32*, const float4*, const u32*, u32, u64*, u32*, u32,
                                                        int, JobStat*, CallState*);
template __global__ void k_update<2, 8, 16, 16, 256, false>(const Job*, const MapDesc*, const u64*, const int*,
                                                        const u32*, const u32*, const float4*, const u32*, u32, u64*, u32*, u32,
                                                        int, JobStat*, CallState*);
template __global__ void k_update<2, 8, 8, 16, 256, false>(const Job*, const MapDesc*, const u64*, const int*,
                                                        const u32*, const u32*, const float4*, const u32*, u32, u64*, u32*, u32,
                                                        int, JobStat*, CallState*);
template __global__ void k_update<2, 4, 8, 16, 256, false>(const Job*, const MapDesc*, const u64*, const int*,
                                                        const u32*, const u32*, const float4*, const u32*, u32, u64*, u32*, u32,
                                                        int, JobStat*, CallState*);
template __global__ void k_update<2, 16, 16, 16, 1024, false>(const Job*, const MapDesc*, const u64*, const int*,
                                                        const u32*, const u32*, const float4*, const u32*, u32, u64*, u32*, u32,
                                                        int, JobStat*, CallState*);
template __global__ void k_update<2, 16, 16, 8, 1024, false>(const Job*, const MapDesc*, const u64*, const int*,
                                                        const u32*, const u32*, const float4*, const u32*, u32, u64*, u32*, u32,
                                                        int, JobStat*, CallState*);
template __global__ void k_update<2, 16, 16, 4, 1024, false>(const Job*, const MapDesc*, const u64*, const int*,
                                                        const u32*, const u32*, const float4*, const u32*, u32, u64*, u32*, u32,
                                                        int, JobStat*, CallState*);
template __global__ void k_update<2, 16, 16, 8, 512, false>(const Job*, const MapDesc*, const u64*, const int*,
                                                        const u32*, const u32*, const float4*, const u32*, u32, u64*, u32*, u32,
                                                        int, JobStat*, CallState*);
template __global__ void k_update<0, 16, 16, 8, 512, true>(const Job*, const MapDesc*, const u64*, const int*,
                                                        const u32*, const u32*, const float4*, const u32*, u32, u64*,
                                                        u32*, u32, int, JobStat*, CallState*);
template __global__ void k_update<1, 16, 16, 8, 512, true>(const Job*, const MapDesc*, const u64*, const int*,
                                                        const u32*, const u32*, const float4*, const u32*, u32, u64*,
                                                        u32*, u32, int, JobStat*, CallState*);
template __global__ void k_update<2, 16, 16, 8, 512, true>(const Job*, const MapDesc*, const u64*, const int*,
                                                        const u32*, const u32*, const float4*, const u32*, u32, u64*,
                                                        u32*, u32, int, JobStat*, CallState*);
template __global__ void k_update<0, 16, 16, 8, 256, true>(const Job*, const MapDesc*, const u64*, const int*,
                                                        const u32*, const u32*, const float4*, const u32*, u32, u64*,
                                                        u32*, u32, int, JobStat*, CallState*);
template __global__ void k_update<0, 16, 16, 4, 256, true>(const Job*, const MapDesc*, const u64*, const int*,
                                                        const u32*, const u32*, const float4*, const u32*, u32, u64*,
                                                        u32*, u32, int, JobStat*, CallState*);
template __global__ void k_update<1, 16, 16, 8, 256, true>(const Job*, const MapDesc*, const u64*, const int*,
                                                        const u32*, const u32*, const float4*, const u32*, u32, u64*,
                                                        u32*, u32, int, JobStat*, CallState*);
template __global__ void k_update<1, 16, 16, 4, 256, true>(const Job*, const MapDesc*, const u64*, const int*,
                                                        const u32*, const u32*, const float4*, const u32*, u32, u64*,
                                                        u32*, u32, int, JobStat*, CallState*);
template __global__ void k_update<2, 16, 16, 8, 256, true>(const Job*, const MapDesc*, const u64*, const int*,
                                                        const u32*, const u32*, const float4*, const u32*, u32, u64*,
                                                        u32*, u32, int, JobStat*, CallState*);
template __global__ void k_update<2, 16, 16, 4, 256, true>(const Job*, const MapDesc*, const u64*, const int*,
                                                        const u32*, const u32*, const float4*, const u32*, u32, u64*,
                                                        u32*, u32, int, JobStat*, CallState*);


// ---------------------------------------------------------------------------
// finish: commit block counts, fold statistics, clean per-call tables
// ---------------------------------------------------------------------------
// The call's last kernel, in one launch: workgroups [0, nmaps) fold each map's statistics,
// workgroups [nmaps, grid) free the per-call block set, and the workgroup that finishes last
// (counted in cs->finish_done) resets the call's counters for the next call.

// Frees the per-call block set: the listed slots, or the whole table after a failed call
// (whose set may hold keys that never reached the list).  Workgroup wg of nwg.
__device__ inline void cleanup_part(u32 wg, u32 nwg, u64* __restrict__ tkeys, u32 tkey_cap,
                                    const u32* __restrict__ tlist, u32 tlist_cap,
                                    const CallState* __restrict__ cs) {
    const u32 stride = nwg * 256u;
    if (cs->error) {
        for (u32 i = wg * 256u + threadIdx.x; i < tkey_cap; i += stride) tkeys[i] = kEmpty;
    } else {
        const u32 nt = cs->t_count < tlist_cap ? cs->t_count : tlist_cap;
        for (u32 i = wg * 256u + threadIdx.x; i < nt; i += stride) tkeys[tlist[i]] = kEmpty;
    }
}

// Map m (one workgroup): folds the call's per-frame statistics into the map, commits its new
// blocks and clears its frames' statistics.
__device__ inline void finish_map(int m, const Job* __restrict__ jobs, const MapDesc* __restrict__ maps,
                                  JobStat* __restrict__ jst, const CallState* __restrict__ cs,
                                  u64* s_acc) {
    MapState* st = maps[m].st;
    const bool ok = st->error == 0 && cs->error == 0;
    if (threadIdx.x < 8) s_acc[threadIdx.x] = 0;
    __syncthreads();
    const int j0 = maps[m].job0, j1 = maps[m].job0 + maps[m].njobs;
    if (ok) {
        u64 a[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        for (int j = j0 + threadIdx.x; j < j1; j += 256) {
            const JobStat& s = jst[j];
            a[0] += jobs[j].n;
            a[1] += s.valid;
            a[2] += s.invalid;
            a[3] += s.oob_pts + s.oob_rays;
            a[4] += s.rays - s.oob_rays;
            a[5] += s.touches;
            a[6] += s.voxels;
            a[7] += s.cells;
        }
        // summed over the wave first (ok is the same for the whole workgroup): one lane adds
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const u64 t = wave_sum64(a[k]);
            if (lane_id() == 0 && t) atomicAdd(&s_acc[k], t);
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        if (ok) {
            st->new_blocks += st->new_count;
            st->block_count += st->new_count;
            st->calls += 1;
            st->points += s_acc[0];
            st->valid += s_acc[1];
            st->invalid += s_acc[2];
            st->oob += s_acc[3];
            st->rays += s_acc[4];
            st->touches += s_acc[5];
            st->voxels += s_acc[6];
            st->cells += s_acc[7];
        }
        if (cs->error != 0 && st->error == 0) st->error = cs->error;
        st->new_count = 0;
    }
    for (int j = j0 + threadIdx.x; j < j1; j += 256) {
        JobStat z;
        z.valid = z.invalid = z.oob_pts = z.oob_rays = z.rays = z.touches = z.voxels = z.cells = 0;
        jst[j] = z;
    }
}

__global__ __launch_bounds__(256) void k_finish_call(const Job* __restrict__ jobs,
                                                     const MapDesc* __restrict__ maps, int nmaps,
                                                     JobStat* __restrict__ jst, u64* __restrict__ tkeys,
                                                     u32 tkey_cap, const u32* __restrict__ tlist,
                                                     u32 tlist_cap, CallState* __restrict__ cs) {
    __shared__ u64 s_acc[8];
    __shared__ bool s_last;
    if ((int)blockIdx.x < nmaps)
        finish_map((int)blockIdx.x, jobs, maps, jst, cs, s_acc);
    else
        cleanup_part(blockIdx.x - (u32)nmaps, gridDim.x - (u32)nmaps, tkeys, tkey_cap, tlist, tlist_cap, cs);
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        s_last = atomicAdd(&cs->finish_done, 1u) == gridDim.x - 1u;
    }
    __syncthreads();
    if (s_last && threadIdx.x == 0) {
        __threadfence();
        cs->ray_count = 0;
        cs->t_count = 0;
        cs->work_next = 0;
        cs->scan_done = 0;
        cs->error = 0;
        cs->finish_done = 0;
    }
}

// ---------------------------------------------------------------------------
// projection mapping (Sec. IV-B): voxels projected into the depth image
// ---------------------------------------------------------------------------
// One workgroup per block of the call's block set (the blocks the frames' truncation bands
// cross), each thread holding 16 voxels in registers and folding, in order, the call's frames of
// its map whose bands cross this block (bins[t * JM + frame] > 0: the crossing counts, cleared
// here for the next call), so that a call of several frames equals one call per frame: the voxel centre goes to camera coordinates and to a pixel (binary32, fixed order,
// no contraction: the same decisions as the point path's), the pixel's point must be valid, and
// a depth difference above -delta updates the voxel by Eqs. (3)-(4) with the weight of Eq. (2)
// or (5).  One observation per voxel and frame: no sums, no atomics.
template <int STORAGE>
__global__ __launch_bounds__(256) void k_project(const Job* __restrict__ jobs, const MapDesc* __restrict__ maps,
                                                 const u64* __restrict__ t_key, const int* __restrict__ t_slot,
                                                 u32* __restrict__ bins, u32 JM,
                                                 Intrinsics K, u64* __restrict__ touch_key,
                                                 u32* __restrict__ touch_n, u32 touch_cap, int keep_touches,
                                                 JobStat* __restrict__ jst, CallState* __restrict__ cs) {
    constexpr int VPT = 16;
    __shared__ u32 lds8[4];
    __shared__ u32 s_tbase;
    const u32 nt = cs->error ? 0u : cs->t_count;
    for (u32 t = blockIdx.x; t < nt; t += gridDim.x) {
        const u64 tk = t_key[t];
        const MapDesc M = maps[(u32)(tk >> 45)];
        if (M.st->error != 0) continue;
        int bx, by, bz;
        unpack_block(tk & ((1ull << 45) - 1), bx, by, bz);
        const int ts = t_slot[t];
        const bool is_new = (ts & 0x40000000) != 0;
        const size_t slot = (size_t)(ts & 0x3FFFFFFF);
        float D[VPT], W[VPT];
        u32 nobs[VPT];
#pragma unroll
        for (int j = 0; j < VPT; ++j) {
            nobs[j] = 0;
            if (is_new) { D[j] = 0.0f; W[j] = 0.0f; }
            else load_voxel<STORAGE>(M.pool, slot * 4096 + threadIdx.x + 256 * j, D[j], W[j]);
        }
        u32 updates = 0;
        for (int f = 0; f < M.njobs; ++f) {
            const u32 nb = bins[(size_t)t * JM + (u32)f];
            __syncthreads();                       // every thread has read the count
            if (threadIdx.x == 0 && nb) bins[(size_t)t * JM + (u32)f] = 0u;
            if (!nb) continue;                     // this frame's bands do not cross the block
            const Job& J = jobs[M.job0 + f];
            const u32 width = J.width, height = J.width ? J.n / J.width : 0u;
            const float s0 = J.pose[3], s1 = J.pose[7], s2 = J.pose[11];
#pragma unroll 4
            for (int j = 0; j < VPT; ++j) {
                const u32 l = threadIdx.x + 256u * (u32)j;
                const int g0 = 16 * bx + (int)(l & 15), g1 = 16 * by + (int)((l >> 4) & 15), g2 = 16 * bz + (int)(l >> 8);
                const float e0 = ((float)g0 + 0.5f) * M.v - s0;
                const float e1 = ((float)g1 + 0.5f) * M.v - s1;
                const float e2 = ((float)g2 + 0.5f) * M.v - s2;
                const float c0 = (J.pose[0] * e0 + J.pose[4] * e1) + J.pose[8] * e2;
                const float c1 = (J.pose[1] * e0 + J.pose[5] * e1) + J.pose[9] * e2;
                const float c2 = (J.pose[2] * e0 + J.pose[6] * e1) + J.pose[10] * e2;
                if (!(c2 > 0.0f)) continue;
                const float uf = K.fx * (c0 / c2) + K.cx;
                const float vf = K.fy * (c1 / c2) + K.cy;
                if (!(uf >= 0.0f && uf < (float)width && vf >= 0.0f && vf < (float)height)) continue;
                const size_t pix = (size_t)__builtin_floorf(uf) + (size_t)width * (size_t)__builtin_floorf(vf);
                const float* pp = J.pts + 3 * pix;
                const float x = pp[0], y = pp[1], z = pp[2];
                float q[3];
                if (classify_point(M, J.pose, x, y, z, q) != 1) continue;
                const float d = z - c2;
                if (!(d > -M.delta)) continue;
                float w = M.weighting == 1 ? 1.0f / (z * z) : 1.0f;
                if (M.weighting == 1) {
                    const float ramp = (d + M.delta) * M.ramp;
                    w = w * (d > -M.eps ? 1.0f : ramp);
                }
                nobs[j] += 1;
                updates += 1;
                if (!(w > 0.0f)) continue;
                float dc = d > M.delta ? M.delta : d;
                if (STORAGE != 0) dc = dc * M.inv_delta;
                float Dn = (W[j] * D[j] + w * dc) / (W[j] + w);
                float Wn = W[j] + w;
                if (Wn > M.w_max) Wn = M.w_max;
                round_to_storage<STORAGE>(Dn, Wn);
                D[j] = Dn;
                W[j] = Wn;
            }
        }
        u32 cells = 0;
#pragma unroll
        for (int j = 0; j < VPT; ++j) {
            store_voxel<STORAGE>(M.pool, slot * 4096 + threadIdx.x + 256 * j, D[j], W[j]);
            cells += nobs[j] ? 1u : 0u;
        }
        if (threadIdx.x == 0 && M.dirty) M.dirty[slot] = 1u;
        const u32 wu = wave_sum(updates), wc = wave_sum(cells);
        if (lane_id() == 0 && wu) {
            atomicAdd(&jst[M.job0].touches, (u64)wu);
            atomicAdd(&jst[M.job0].voxels, (u64)wu);
            atomicAdd(&jst[M.job0].cells, (u64)wc);
        }
        if (keep_touches) {
            u32 tot;
            const u32 incl = block_scan<256>(cells, lds8, &tot);
            if (threadIdx.x == 0) s_tbase = atomicAdd(&cs->touch_count, tot);
            __syncthreads();
            u32 pos = s_tbase + incl - cells;
#pragma unroll
            for (int j = 0; j < VPT; ++j) {
                if (nobs[j]) {
                    const u32 l = threadIdx.x + 256u * (u32)j;
                    if (pos < touch_cap) {
                        touch_key[pos] = ((u64)M.map_id << 57) |
                                         voxel_key_of(16 * bx + (int)(l & 15), 16 * by + (int)((l >> 4) & 15),
                                                      16 * bz + (int)(l >> 8));
                        touch_n[pos] = nobs[j];
                    }
                    pos++;
                }
            }
        }
        __syncthreads();
    }
}
template __global__ void k_project<0>(const Job*, const MapDesc*, const u64*, const int*, u32*, u32, Intrinsics,
                                      u64*, u32*, u32, int, JobStat*, CallState*);
template __global__ void k_project<1>(const Job*, const MapDesc*, const u64*, const int*, u32*, u32, Intrinsics,
                                      u64*, u32*, u32, int, JobStat*, CallState*);
template __global__ void k_project<2>(const Job*, const MapDesc*, const u64*, const int*, u32*, u32, Intrinsics,
                                      u64*, u32*, u32, int, JobStat*, CallState*);

// ---------------------------------------------------------------------------
// query: trilinear interpolation of the distance field (the accuracy evaluation, Sec. VI-A)
// ---------------------------------------------------------------------------
// Voxel (i, j, k) holds the field at its centre ((i, j, k) + 1/2) v.  A query point q takes the
// eight voxels around it: u = q * (1/v) - 1/2 per axis (binary32, with the map's binary32
// reciprocal of v), base corner floor(u), fractions f = u - floor(u); the distance is the
// trilinear blend of the eight corner distances, along x, then y, then z (binary32).  It is
// known only where all eight voxels are allocated and observed (W > 0); elsewhere the output is
// NaN.  One thread per query; corners in the block of the previous corner reuse its lookup.

template <int STORAGE>
__global__ __launch_bounds__(256) void k_interpolate(const MapDesc M, const float* __restrict__ q, u32 n,
                                                     float* __restrict__ out) {
    for (u32 i = blockIdx.x * 256u + threadIdx.x; i < n; i += gridDim.x * 256u) {
        int b[3];
        float f[3];
        bool ok = true;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const float u = q[3 * (size_t)i + k] * M.iv - 0.5f;
            const float fl = __builtin_floorf(u);
            ok = ok && fl >= -(float)kVoxLimit && fl < (float)(kVoxLimit - 1);   // false for NaN
            b[k] = ok ? (int)fl : 0;
            f[k] = u - fl;
        }
        float d[8];
        u64 last = kEmpty;
        int slot = -1;
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            d[c] = 0.0f;
            if (!ok) continue;
            const int gx = b[0] + (c & 1), gy = b[1] + ((c >> 1) & 1), gz = b[2] + (c >> 2);
            const u64 bk = block_key_of(gx, gy, gz);
            if (bk != last) {
                slot = find_block(M, bk);
                last = bk;
            }
            if (slot < 0) {
                ok = false;
                continue;
            }
            float D, W;
            load_voxel<STORAGE>(M.pool, (size_t)slot * 4096 + local_of(gx, gy, gz), D, W);
            if (!(W > 0.0f)) ok = false;
            d[c] = STORAGE == 0 ? D : D * M.delta;
        }
        const float gx = 1.0f - f[0], gy = 1.0f - f[1], gz = 1.0f - f[2];
        const float c00 = d[0] * gx + d[1] * f[0];
        const float c10 = d[2] * gx + d[3] * f[0];
        const float c01 = d[4] * gx + d[5] * f[0];
        const float c11 = d[6] * gx + d[7] * f[0];
        const float c0 = c00 * gy + c10 * f[1];
        const float c1 = c01 * gy + c11 * f[1];
        out[i] = ok ? c0 * gz + c1 * f[2] : __builtin_nanf("");
    }
}
template __global__ void k_interpolate<0>(const MapDesc, const float*, u32, float*);
template __global__ void k_interpolate<1>(const MapDesc, const float*, u32, float*);
template __global__ void k_interpolate<2>(const MapDesc, const float*, u32, float*);

// ---------------------------------------------------------------------------
// verification: traversal of voxel-space segments
// ---------------------------------------------------------------------------
__global__ void k_debug_traverse(const float* __restrict__ A, const float* __restrict__ B, int n,
                                 int* __restrict__ out, int cap, int* __restrict__ counts) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float a[3] = {A[3 * i], A[3 * i + 1], A[3 * i + 2]};
    const float b[3] = {B[3 * i], B[3 * i + 1], B[3 * i + 2]};
    for (int k = 0; k < 3; ++k) {
        if (!(a[k] >= -(float)kVoxLimit && a[k] < (float)kVoxLimit && b[k] >= -(float)kVoxLimit &&
              b[k] < (float)kVoxLimit)) {
            counts[i] = -1;   // outside the addressable voxel range
            return;
        }
    }
    Walk w;
    walk_setup_vox(a, b, w);
    int c = 0;
    for (;;) {
        if (c < cap) {
            out[(size_t)i * cap * 3 + 3 * c] = w.g[0];
            out[(size_t)i * cap * 3 + 3 * c + 1] = w.g[1];
            out[(size_t)i * cap * 3 + 3 * c + 2] = w.g[2];
        }
        c++;
        if (w.left == 0) break;
        walk_step(w);
    }
    counts[i] = c;
}

// The blocks of the same traversals, from the block-changing steps alone (as the crossing
// kernel finds them): out[i][c] = block indices, counts[i] = the number of blocks.
__global__ void k_debug_traverse_blocks(const float* __restrict__ A, const float* __restrict__ B, int n,
                                        int* __restrict__ out, int cap, int* __restrict__ counts) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float a[3] = {A[3 * i], A[3 * i + 1], A[3 * i + 2]};
    const float b[3] = {B[3 * i], B[3 * i + 1], B[3 * i + 2]};
    for (int k = 0; k < 3; ++k) {
        if (!(a[k] >= -(float)kVoxLimit && a[k] < (float)kVoxLimit && b[k] >= -(float)kVoxLimit &&
              b[k] < (float)kVoxLimit)) {
            counts[i] = -1;   // outside the addressable voxel range
            return;
        }
    }
    Walk w;
    walk_setup_vox(a, b, w);
    BlockWalk bw;
    block_walk_init(w, bw);
    int c = 0;
    for (int axis = 0; axis >= 0; axis = block_walk_next(bw)) {
        if (c < cap) {
            out[(size_t)i * cap * 3 + 3 * c] = bw.b[0];
            out[(size_t)i * cap * 3 + 3 * c + 1] = bw.b[1];
            out[(size_t)i * cap * 3 + 3 * c + 2] = bw.b[2];
        }
        c++;
    }
    counts[i] = c;
}

}  // namespace vbx
