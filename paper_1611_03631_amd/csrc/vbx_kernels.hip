// HIP kernels of the vbx TSDF integrator (gfx950, wave64).
//
// One integration call runs this pipeline on the map's stream:
//   points   : validity, pose transform, voxel keying (one thread per point, coalesced
//              12-byte loads).  Per-point raycasting writes one ray per valid point.
//              Grouped raycasting (Sec. IV-B) first merges the points of a tile in an LDS
//              hash by voxel, then merges the tile partials of one (frame, voxel) in a
//              global table, all in exact integer sums, and casts one ray per group.
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

__global__ void k_fill_u64(u64* p, u64 val, size_t n) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = val;
}
__global__ void k_fill_u32(u32* p, u32 val, size_t n) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = val;
}
__global__ void k_clear_groups(GroupEntry* t, size_t n) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        GroupEntry e;
        e.key = kEmpty; e.so = 0; e.sq[0] = e.sq[1] = e.sq[2] = 0;
        e.sqhi[0] = e.sqhi[1] = e.sqhi[2] = 0; e.n = 0; e.idx = 0; e.pad = 0;
        t[i] = e;
    }
}
__global__ void k_set_u32(u32* p, u32 v) { *p = v; }

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

// ---------------------------------------------------------------------------
// points: per-point raycasting
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_points_simple(const Job* __restrict__ jobs, int njobs,
                                                       int job_base,
                                                       const MapDesc* __restrict__ maps,
                                                       float4* __restrict__ rays_p,
                                                       u32* __restrict__ rays_job,
                                                       JobStat* __restrict__ jst,
                                                       CallState* __restrict__ cs, u32 ray_cap) {
    __shared__ u32 s_cnt[3];   // valid, invalid, out of bounds
    __shared__ u32 s_base;
    __shared__ u32 lds8[4];
    const int jloc = job_of_tile(jobs, njobs, blockIdx.x);
    const int jid = job_base + jloc;
    const Job& J = jobs[jloc];
    const MapDesc& M = maps[J.map];
    if (threadIdx.x < 3) s_cnt[threadIdx.x] = 0;
    __syncthreads();
    const u32 first = (blockIdx.x - J.tile0) * kTileSimple;
    float q[4][3];
    u32 valid_mask = 0;
    u32 n_inv = 0, n_oob = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        u32 i = first + threadIdx.x + 256u * j;
        if (i < J.n) {
            const float x = J.pts[3 * (size_t)i], y = J.pts[3 * (size_t)i + 1], z = J.pts[3 * (size_t)i + 2];
            int c = classify_point(M, J.pose, x, y, z, q[j]);
            if (c == 1) valid_mask |= 1u << j;
            else if (c == 0) n_inv++;
            else n_oob++;
        }
    }
    u32 nv = __builtin_popcount(valid_mask);
    u32 tot;
    u32 incl = block_scan_256(nv, lds8, &tot);
    if (n_inv) atomicAdd(&s_cnt[1], n_inv);
    if (n_oob) atomicAdd(&s_cnt[2], n_oob);
    if (threadIdx.x == 0) s_base = tot ? atomicAdd(&cs->ray_count, tot) : 0;
    __syncthreads();
    u32 pos = s_base + incl - nv;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        if (valid_mask & (1u << j)) {
            if (pos < ray_cap) {
                // per-point weight: Eq. (2) 1, or the 1/z^2 factor of Eq. (5)
                const float z = J.pts[3 * (size_t)(first + threadIdx.x + 256u * j) + 2];
                float wgt = M.weighting == 1 ? 1.0f / (z * z) : 1.0f;
                rays_p[pos] = make_float4(q[j][0], q[j][1], q[j][2], wgt);
                rays_job[pos] = (u32)jid;
            }
            pos++;
        }
    }
    if (threadIdx.x == 0) {
        if (tot) atomicAdd(&jst[jid].valid, (u64)tot);
        if (s_cnt[1]) atomicAdd(&jst[jid].invalid, (u64)s_cnt[1]);
        if (s_cnt[2]) atomicAdd(&jst[jid].oob_pts, (u64)s_cnt[2]);
        if (tot) atomicAdd(&jst[jid].rays, (u64)tot);
    }
}

// ---------------------------------------------------------------------------
// points: grouped raycasting, tile-level merge in LDS then global merge
// ---------------------------------------------------------------------------
// Fixed-point terms of one point for the exact group mean:
//   Q_k = min(rint(q_k 2^20), 2^20 - 1) with q_k = f_k - floor(f_k), f_k = p_k / v (binary32),
//   Omega = rint(w 2^wbits) (w = 1/z^2) or 1.
__device__ inline void group_terms(const MapDesc& M, const float q[3], float z, int g[3], u32 Q[3],
                                   u64& om) {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        float f = q[k] * M.iv;
        float fl = __builtin_floorf(f);
        g[k] = (int)fl;
        float fr = f - (float)g[k];
        float qs = __builtin_rintf(__builtin_ldexpf(fr, 20));
        u32 Qk = (u32)qs;
        Q[k] = Qk > (1u << 20) - 1 ? (1u << 20) - 1 : Qk;
    }
    if (M.wbits > 0) {
        float w = 1.0f / (z * z);
        om = (u64)__builtin_rintf(__builtin_ldexpf(w, M.wbits));
    } else {
        om = 1;
    }
}

__global__ __launch_bounds__(256) void k_points_grouped(const Job* __restrict__ jobs, int njobs,
                                                        int job_base,
                                                        const MapDesc* __restrict__ maps,
                                                        GroupEntry* __restrict__ table, u32 tmask,
                                                        u32* __restrict__ occ,
                                                        JobStat* __restrict__ jst,
                                                        CallState* __restrict__ cs) {
    __shared__ u64 s_key[kGroupSlots];
    __shared__ u64 s_so[kGroupSlots];
    __shared__ u64 s_sq[3][kGroupSlots];
    __shared__ u32 s_n[kGroupSlots];
    __shared__ u32 s_idx[kGroupSlots];
    __shared__ u32 s_new[kTileGrouped];   // table entries this tile created
    __shared__ u32 s_nnew, s_occ_base;
    __shared__ u32 s_cnt[3];
    const int jloc = job_of_tile(jobs, njobs, blockIdx.x);
    const int jid = job_base + jloc;
    const Job& J = jobs[jloc];
    const MapDesc& M = maps[J.map];
    for (int i = threadIdx.x; i < kGroupSlots; i += 256) {
        s_key[i] = kEmpty; s_so[i] = 0; s_sq[0][i] = 0; s_sq[1][i] = 0; s_sq[2][i] = 0; s_n[i] = 0;
    }
    if (threadIdx.x < 3) s_cnt[threadIdx.x] = 0;
    if (threadIdx.x == 0) s_nnew = 0;
    __syncthreads();

    const u32 tile = blockIdx.x - J.tile0;
    u32 n_valid = 0, n_inv = 0, n_oob = 0;
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        u32 i;
        bool in;
        if (J.width > 0) {
            const u32 tiles_x = (J.width + kTileGroupedW - 1) / kTileGroupedW;
            const u32 ty = tile / tiles_x, tx = tile - ty * tiles_x;
            const u32 col = tx * kTileGroupedW + (threadIdx.x & 31);
            const u32 row = ty * kTileGroupedH + (threadIdx.x >> 5) + 8u * j;
            in = col < J.width && (size_t)row * J.width + col < J.n;
            i = row * J.width + col;
        } else {
            i = tile * kTileGrouped + threadIdx.x + 256u * j;
            in = i < J.n;
        }
        if (!in) continue;
        const float x = J.pts[3 * (size_t)i], y = J.pts[3 * (size_t)i + 1], z = J.pts[3 * (size_t)i + 2];
        float q[3];
        int c = classify_point(M, J.pose, x, y, z, q);
        if (c != 1) { if (c == 0) n_inv++; else n_oob++; continue; }
        n_valid++;
        int g[3];
        u32 Q[3];
        u64 om;
        group_terms(M, q, z, g, Q, om);
        const u64 key = voxel_key_of(g[0], g[1], g[2]);
        u32 h = (u32)mix64(key) & (kGroupSlots - 1);
        for (;;) {
            u64 old = atomicCAS(&s_key[h], kEmpty, key);
            if (old == kEmpty || old == key) break;
            h = (h + 1) & (kGroupSlots - 1);
        }
        atomicAdd(&s_so[h], om);
        atomicAdd(&s_sq[0][h], om * Q[0]);
        atomicAdd(&s_sq[1][h], om * Q[1]);
        atomicAdd(&s_sq[2][h], om * Q[2]);
        atomicAdd(&s_n[h], 1u);
        s_idx[h] = i;
    }
    if (n_valid) atomicAdd(&s_cnt[0], n_valid);
    if (n_inv) atomicAdd(&s_cnt[1], n_inv);
    if (n_oob) atomicAdd(&s_cnt[2], n_oob);
    __syncthreads();

    // merge the tile's partial groups into the global table of this chunk of frames; new
    // table entries are listed in LDS and appended to the occupied list with one atomic
    const u64 tag = (u64)jloc << 57;
    for (int s = threadIdx.x; s < kGroupSlots; s += 256) {
        const u64 key = s_key[s];
        if (key == kEmpty) continue;
        const u64 gk = tag | key;
        u32 h = (u32)mix64(gk) & tmask;
        for (;;) {
            u64 old = atomicCAS(&table[h].key, kEmpty, gk);
            if (old == kEmpty) { s_new[atomicAdd(&s_nnew, 1u)] = h; break; }
            if (old == gk) break;
            h = (h + 1) & tmask;
        }
        GroupEntry* E = &table[h];
        atomicAdd(&E->so, s_so[s]);
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const u64 add = s_sq[k][s];
            const u64 old = atomicAdd(&E->sq[k], add);
            if (old + add < old) atomicAdd(&E->sqhi[k], 1u);   // carry into the high word
        }
        const u32 n = s_n[s];
        atomicAdd(&E->n, n);
        if (n == 1) E->idx = s_idx[s];
    }
    __syncthreads();
    if (threadIdx.x == 0) s_occ_base = s_nnew ? atomicAdd(&cs->occ_count, s_nnew) : 0u;
    __syncthreads();
    for (u32 k = threadIdx.x; k < s_nnew; k += 256) occ[s_occ_base + k] = s_new[k];
    if (threadIdx.x == 0) {
        if (s_cnt[0]) atomicAdd(&jst[jid].valid, (u64)s_cnt[0]);
        if (s_cnt[1]) atomicAdd(&jst[jid].invalid, (u64)s_cnt[1]);
        if (s_cnt[2]) atomicAdd(&jst[jid].oob_pts, (u64)s_cnt[2]);
    }
}

// One ray per group: its end point is the exact weighted mean (singletons keep the point),
// its weight the group's summed weight.  Cleans the table entry for the next chunk.
__global__ __launch_bounds__(256) void k_groups_to_rays(const Job* __restrict__ jobs, int job_base,
                                                        const MapDesc* __restrict__ maps,
                                                        GroupEntry* __restrict__ table,
                                                        const u32* __restrict__ occ,
                                                        float4* __restrict__ rays_p,
                                                        u32* __restrict__ rays_job,
                                                        JobStat* __restrict__ jst,
                                                        CallState* __restrict__ cs, u32 ray_cap) {
    __shared__ u32 lds8[4];
    __shared__ u32 s_base;
    const u32 nocc = cs->occ_count;
    for (u32 base = blockIdx.x * 256u; base < nocc; base += gridDim.x * 256u) {
        const u32 i = base + threadIdx.x;
        const bool act = i < nocc;
        float4 ray = make_float4(0.f, 0.f, 0.f, 0.f);
        u32 jid = 0;
        if (act) {
            const u32 h = occ[i];
            GroupEntry E = table[h];
            const u32 jloc = (u32)(E.key >> 57);
            jid = job_base + jloc;
            const Job& J = jobs[jloc];
            const MapDesc& M = maps[J.map];
            int g[3];
            unpack_voxel(E.key & ((1ull << 57) - 1), g[0], g[1], g[2]);
            float p[3];
            if (E.n == 1) {
                const float x = J.pts[3 * (size_t)E.idx], y = J.pts[3 * (size_t)E.idx + 1],
                            z = J.pts[3 * (size_t)E.idx + 2];
                classify_point(M, J.pose, x, y, z, p);
            } else {
                const double den = (double)E.so * 1048576.0;
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    const double hi = (double)(u64)E.sqhi[k];
                    const double lo = (double)E.sq[k];
                    const double m = (hi * 18446744073709551616.0 + lo) / den;
                    p[k] = (float)(((double)g[k] + m) * (double)M.v);
                }
            }
            const float wgt = M.wbits > 0 ? (float)((double)E.so * __builtin_ldexp(1.0, -M.wbits))
                                          : (float)E.n;
            ray = make_float4(p[0], p[1], p[2], wgt);
            GroupEntry Z;
            Z.key = kEmpty; Z.so = 0; Z.sq[0] = Z.sq[1] = Z.sq[2] = 0;
            Z.sqhi[0] = Z.sqhi[1] = Z.sqhi[2] = 0; Z.n = 0; Z.idx = 0; Z.pad = 0;
            table[h] = Z;
        }
        u32 tot;
        const u32 incl = block_scan_256(act ? 1u : 0u, lds8, &tot);
        if (threadIdx.x == 0) s_base = atomicAdd(&cs->ray_count, tot);
        __syncthreads();
        if (act) {
            const u32 pos = s_base + incl - 1;
            if (pos < ray_cap) { rays_p[pos] = ray; rays_job[pos] = jid; }
        }
        // per-frame ray counts, aggregated per wave
        {
            u64 pending = __ballot(act);
            const int lane = lane_id();
            while (pending) {
                int leader = __ffsll((long long)pending) - 1;
                u32 k = __shfl(jid, leader);
                u64 grp = __ballot(((pending >> lane) & 1ull) && jid == k);
                if (lane == leader) atomicAdd(&jst[k].rays, (u64)__popcll(grp));
                pending &= ~grp;
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// cross: walk the band of each ray, record (block, ray) crossings
// ---------------------------------------------------------------------------
// Inserts a (map, block) key into the per-call block set; returns its slot.
__device__ inline u32 tset_insert(u64* tkeys, u32 tmask, u64 key, u32* tlist, u32 tlist_cap,
                                  CallState* cs) {
    u32 h = (u32)mix64(key) & tmask;
    for (u32 probe = 0; probe <= tmask; ++probe) {
        u64 old = atomicCAS(&tkeys[h], kEmpty, key);
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

// Per workgroup of 256 rays, in three phases separated by barriers:
//  1. walk every ray, count its block crossings and enter the block keys in an LDS set;
//  2. insert each distinct block of the workgroup once into the per-call block set;
//  3. walk again and write the crossings at a range reserved with one global atomic.
constexpr int kCrossSlots = 2048;   // LDS block-key set (at most 256 rays x 7 blocks)

__device__ inline u32 lds_set_insert(u64* keys, u64 key) {
    u32 h = (u32)mix64(key) & (kCrossSlots - 1);
    for (;;) {
        const u64 old = atomicCAS(&keys[h], kEmpty, key);
        if (old == kEmpty || old == key) return h;
        h = (h + 1) & (kCrossSlots - 1);
    }
}
__device__ inline u32 lds_set_find(const u64* keys, u64 key) {
    u32 h = (u32)mix64(key) & (kCrossSlots - 1);
    while (keys[h] != key) h = (h + 1) & (kCrossSlots - 1);
    return h;
}

__global__ __launch_bounds__(256) void k_cross(const Job* __restrict__ jobs,
                                               const MapDesc* __restrict__ maps,
                                               const float4* __restrict__ rays_p,
                                               const u32* __restrict__ rays_job,
                                               u64* __restrict__ tkeys, u32 tmask,
                                               u32* __restrict__ tlist, u32 tlist_cap,
                                               uint2* __restrict__ cross, u32 cross_cap,
                                               JobStat* __restrict__ jst,
                                               CallState* __restrict__ cs, u32 ray_cap) {
    __shared__ u64 s_key[kCrossSlots];
    __shared__ u32 s_h[kCrossSlots];
    __shared__ u32 lds8[4];
    __shared__ u32 s_base;
    const u32 nrays = cs->ray_count < ray_cap ? cs->ray_count : ray_cap;
    for (u32 base = blockIdx.x * 256u; base < nrays; base += gridDim.x * 256u) {
        for (int i = threadIdx.x; i < kCrossSlots; i += 256) s_key[i] = kEmpty;
        __syncthreads();
        const u32 i = base + threadIdx.x;
        bool ok = false;
        u32 jid = 0;
        float p[3] = {0.f, 0.f, 0.f}, s[3] = {0.f, 0.f, 0.f};
        u64 mapbits = 0;
        const MapDesc* Mp = maps;
        if (i < nrays) {
            jid = rays_job[i];
            const Job& J = jobs[jid];
            Mp = &maps[J.map];
            const float4 rp = rays_p[i];
            p[0] = rp.x; p[1] = rp.y; p[2] = rp.z;
            s[0] = J.pose[3]; s[1] = J.pose[7]; s[2] = J.pose[11];
            mapbits = (u64)Mp->map_id << 45;
            float e[3], r;
            Walk w;
            ok = walk_setup(*Mp, p, s, e, r, w);
        }
        // phase 1
        u32 ncross = 0;
        if (ok) {
            float e[3], r;
            Walk w;
            walk_setup(*Mp, p, s, e, r, w);
            u64 cur = kEmpty;
            for (int guard = 0; guard < kMaxStepsPerRay; ++guard) {
                const u64 bk = block_key_of(w.g[0], w.g[1], w.g[2]);
                if (bk != cur) {
                    cur = bk;
                    lds_set_insert(s_key, mapbits | bk);
                    ncross++;
                }
                if (w.left == 0) break;
                walk_step(w);
            }
        }
        u32 tot;
        const u32 incl = block_scan_256(ncross, lds8, &tot);
        if (threadIdx.x == 0) {
            const u32 b0 = atomicAdd(&cs->cross_count, tot);
            if ((u64)b0 + tot > cross_cap) cs->error = -4;
            s_base = b0;
        }
        // phase 2
        for (int k = threadIdx.x; k < kCrossSlots; k += 256) {
            const u64 key = s_key[k];
            if (key != kEmpty) s_h[k] = tset_insert(tkeys, tmask, key, tlist, tlist_cap, cs);
        }
        __syncthreads();
        // phase 3
        if (ok) {
            u32 pos = s_base + incl - ncross;
            float e[3], r;
            Walk w;
            walk_setup(*Mp, p, s, e, r, w);
            u64 cur = kEmpty;
            for (int guard = 0; guard < kMaxStepsPerRay; ++guard) {
                const u64 bk = block_key_of(w.g[0], w.g[1], w.g[2]);
                if (bk != cur) {
                    cur = bk;
                    const u32 h = s_h[lds_set_find(s_key, mapbits | bk)];
                    if (pos < cross_cap && h != 0xFFFFFFFFu) cross[pos] = make_uint2(h, i);
                    pos++;
                }
                if (w.left == 0) break;
                walk_step(w);
            }
        }
        // out-of-bounds rays per frame (rare); rays were counted when created
        const bool oob = i < nrays && !ok;
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
// The 64 lanes of a wave read 64 consecutive slots of the probe sequence at once and vote
// for a match or a free slot.  Keys are never deleted, so a key is absent when a free slot
// comes before any match.  Returns the slot index holding key, or -1 (with *free_at set to
// the first free slot of the probe sequence).  Wave-uniform arguments and result.
__device__ inline int coop_find(const u64* __restrict__ hkeys, u32 hmask, u64 key, u32* free_at) {
    const int lane = lane_id();
    const u32 start = (u32)mix64(key) & hmask;
    for (u32 base = 0; base <= hmask; base += 64) {
        const u32 slot = (start + base + lane) & hmask;
        const u64 k = hkeys[slot];
        const u64 match = __ballot(k == key);
        const u64 empty = __ballot(k == kEmpty);
        const int fm = match ? __ffsll((long long)match) : 65;
        const int fe = empty ? __ffsll((long long)empty) : 65;
        if (fm < fe) return (int)((start + base + fm - 1) & hmask);
        if (fe < 65) { *free_at = (start + base + fe - 1) & hmask; return -1; }
    }
    *free_at = 0xFFFFFFFFu;
    return -1;
}

__global__ __launch_bounds__(256) void k_resolve(const MapDesc* __restrict__ maps,
                                                 const u64* __restrict__ tkeys,
                                                 u32* __restrict__ tval,
                                                 const u32* __restrict__ tlist,
                                                 u64* __restrict__ t_key, int* __restrict__ t_slot,
                                                 CallState* __restrict__ cs) {
    const u32 nt = cs->error ? 0u : cs->t_count;
    const int lane = lane_id();
    const u32 wave_global = (blockIdx.x * 256u + threadIdx.x) >> 6;
    const u32 nwaves = (gridDim.x * 256u) >> 6;
    for (u32 wbase = wave_global * 64u; wbase < nt; wbase += nwaves * 64u) {
        const u32 i = wbase + lane;
        u64 key = kEmpty;
        if (i < nt) {
            const u32 h = tlist[i];
            key = tkeys[h];
            tval[h] = i;
            t_key[i] = key;
        }
        int my_slot = -1;
        u64 act = __ballot(i < nt);
        while (act) {
            const int l = __ffsll((long long)act) - 1;
            act &= act - 1;
            const u64 k = __shfl(key, l);
            const MapDesc& M = maps[(u32)(k >> 45)];
            u32 free_at;
            const int pos = coop_find(M.hkeys, M.hmask, k & ((1ull << 45) - 1), &free_at);
            const int slot = pos >= 0 ? M.hslots[pos] : -1;
            if (lane == l) my_slot = slot;
        }
        if (i < nt) {
            if (my_slot >= 0) {
                t_slot[i] = my_slot;
            } else {
                const MapDesc& M = maps[(u32)(key >> 45)];
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
    const u32 wave_global = (blockIdx.x * 256u + threadIdx.x) >> 6;
    const u32 nwaves = (gridDim.x * 256u) >> 6;
    for (u32 wbase = wave_global * 64u; wbase < nt; wbase += nwaves * 64u) {
        const u32 i = wbase + lane;
        bool pending = false;
        u64 key = kEmpty;
        int slot = 0;
        if (i < nt) {
            key = t_key[i];
            const int s = t_slot[i];
            if (s <= -2) {
                const MapDesc& M = maps[(u32)(key >> 45)];
                MapState* st = M.st;
                const u32 rank = (u32)(-s - 2);
                if (st->error == 0 && (u64)st->block_count + st->new_count <= M.capacity && cs->error == 0) {
                    pending = true;
                    slot = (int)(st->block_count + rank);
                } else {
                    if (cs->error == 0) st->error = -3;   // VBX_ERR_POOL_FULL, map left unchanged
                }
            }
        }
        u64 act = __ballot(pending);
        while (act) {
            const int l = __ffsll((long long)act) - 1;
            act &= act - 1;
            const u64 k = __shfl(key, l);
            const int sl = __shfl(slot, l);
            const MapDesc& M = maps[(u32)(k >> 45)];
            const u64 bk = k & ((1ull << 45) - 1);
            for (;;) {
                u32 free_at;
                const int pos = coop_find(M.hkeys, M.hmask, bk, &free_at);
                if (pos >= 0 || free_at == 0xFFFFFFFFu) break;   // present (cannot happen) or full
                u64 old = 0;
                if (lane == 0) old = atomicCAS(&M.hkeys[free_at], kEmpty, bk);
                old = __shfl(old, 0);
                if (old == kEmpty) {
                    if (lane == 0) M.hslots[free_at] = sl;
                    break;
                }
            }
        }
        if (pending) t_slot[i] = slot | (int)0x40000000;   // bit 30: new block
    }
}

// ---------------------------------------------------------------------------
// bins: counting sort of crossings by (block, frame)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_bin_count(const Job* __restrict__ jobs,
                                                   const uint2* __restrict__ cross,
                                                   const u32* __restrict__ tval,
                                                   const u32* __restrict__ rays_job,
                                                   u32* __restrict__ bins, u32 JM,
                                                   CallState* __restrict__ cs) {
    const u32 nc = cs->error ? 0u : cs->cross_count;
    for (u32 base = blockIdx.x * 256u; base < nc; base += gridDim.x * 256u) {
        const u32 i = base + threadIdx.x;
        u32 b = 0;
        if (i < nc) {
            const uint2 c = cross[i];
            b = tval[c.x] * JM + jobs[rays_job[c.y]].jm;
        }
        wave_count_by_key(bins, i < nc, b);
    }
}

// Exclusive scan of bins[0, n) with n = t_count * JM, in chunks of 4096 (16 per thread).
constexpr int kScanChunk = 4096;

__global__ __launch_bounds__(256) void k_scan_sums(const u32* __restrict__ bins, u32 JM,
                                                   u32* __restrict__ partial,
                                                   const CallState* __restrict__ cs) {
    __shared__ u32 lds8[4];
    const u32 n = cs->error ? 0u : cs->t_count * JM;
    const u32 base = blockIdx.x * (u32)kScanChunk;
    u32 s = 0;
    if (base < n) {
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            const u32 i = base + threadIdx.x * 16u + j;
            if (i < n) s += bins[i];
        }
    }
    u32 tot;
    block_scan_256(s, lds8, &tot);
    if (threadIdx.x == 0) partial[blockIdx.x] = tot;
}

__global__ __launch_bounds__(256) void k_scan_partials(u32* __restrict__ partial, u32 nparts,
                                                       u32* __restrict__ off, u32 JM,
                                                       const CallState* __restrict__ cs) {
    __shared__ u32 lds8[4];
    const u32 n = cs->error ? 0u : cs->t_count * JM;
    const u32 used = (n + kScanChunk - 1) / kScanChunk;
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

__global__ __launch_bounds__(256) void k_scan_final(const u32* __restrict__ bins,
                                                    const u32* __restrict__ partial,
                                                    u32* __restrict__ off, u32 JM,
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
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        const u32 i = base + threadIdx.x * 16u + j;
        if (i < n) off[i] = run;
        run += v[j];
    }
}

// Copies each crossing's ray (end point, weight) to its bin position, so that the update
// kernel reads every (block, frame) bin contiguously.  Counts are decremented back to zero,
// leaving the bins clean for the next call.
__global__ __launch_bounds__(256) void k_scatter(const Job* __restrict__ jobs,
                                                 const uint2* __restrict__ cross,
                                                 const u32* __restrict__ tval,
                                                 const u32* __restrict__ rays_job,
                                                 u32* __restrict__ bins, const u32* __restrict__ off,
                                                 u32 JM, const float4* __restrict__ rays_p,
                                                 float4* __restrict__ sorted,
                                                 CallState* __restrict__ cs) {
    const u32 nc = cs->error ? 0u : cs->cross_count;
    const int lane = lane_id();
    for (u32 base = blockIdx.x * 256u; base < nc; base += gridDim.x * 256u) {
        const u32 i = base + threadIdx.x;
        const bool act = i < nc;
        u32 b = 0, ray = 0;
        if (act) {
            const uint2 c = cross[i];
            ray = c.y;
            b = tval[c.x] * JM + jobs[rays_job[ray]].jm;
        }
        // lanes sharing a bin take consecutive positions reserved by one atomic
        u64 pending = __ballot(act);
        u32 pos = 0;
        while (pending) {
            const int leader = __ffsll((long long)pending) - 1;
            const u32 kb = __shfl(b, leader);
            const bool mine = ((pending >> lane) & 1ull) && b == kb;
            const u64 grp = __ballot(mine);
            u32 old = 0;
            if (lane == leader) old = atomicSub(&bins[kb], (u32)__popcll(grp));
            old = __shfl(old, leader);
            if (mine) {
                const u32 rank = (u32)__popcll(grp & ((1ull << lane) - 1ull));
                pos = off[kb] + old - 1u - rank;
            }
            pending &= ~grp;
        }
        if (act) sorted[pos] = rays_p[ray];
    }
}

// ---------------------------------------------------------------------------
// update: one workgroup per touched block
// ---------------------------------------------------------------------------
template <int STORAGE>
__device__ inline void load_voxel(const void* pool, size_t idx, float& D, float& W) {
    if (STORAGE == 0) {
        const float2 dw = ((const float2*)pool)[idx];
        D = dw.x; W = dw.y;
    } else {
        const u32 raw = ((const u32*)pool)[idx];
        D = __half2float(__ushort_as_half((unsigned short)(raw & 0xFFFF)));
        W = __half2float(__ushort_as_half((unsigned short)(raw >> 16)));
    }
}
template <int STORAGE>
__device__ inline void store_voxel(void* pool, size_t idx, float D, float W) {
    if (STORAGE == 0) {
        ((float2*)pool)[idx] = make_float2(D, W);
    } else {
        const u32 d = __half_as_ushort(__float2half_rn(D));
        const u32 w = __half_as_ushort(__float2half_rn(W));
        ((u32*)pool)[idx] = d | (w << 16);
    }
}

constexpr int kOffWindow = 256;   // frames whose bin offsets are staged in LDS at a time

// Work item u = t * SPLIT + q: slab q (local z in [q*16/SPLIT, (q+1)*16/SPLIT)) of touched block t.
// Slabs of one block are independent (different voxels) and replay the same rays, so a
// block's frames run in parallel across SPLIT workgroups with 1/SPLIT of the LDS each.
template <int STORAGE, int SPLIT>
__global__ __launch_bounds__(256) void k_update(const Job* __restrict__ jobs,
                                                const MapDesc* __restrict__ maps,
                                                const u64* __restrict__ t_key,
                                                const int* __restrict__ t_slot,
                                                const u32* __restrict__ off,
                                                const float4* __restrict__ sorted, u32 JM,
                                                u64* __restrict__ touch_key,
                                                u32* __restrict__ touch_n, u32 touch_cap,
                                                int keep_touches,
                                                JobStat* __restrict__ jst,
                                                CallState* __restrict__ cs) {
    constexpr int VOX = 4096 / SPLIT;      // voxels of one slab
    constexpr int VPT = VOX / 256;         // voxels per thread
    constexpr int ZS = 16 / SPLIT;         // slab thickness
    __shared__ u64 a_w[VOX];    // sum of fixed-point weights
    __shared__ u64 a_d[VOX];    // sum of fixed-point weight * distance/delta (two's complement)
    __shared__ u32 a_n[VOX];    // rays
    __shared__ u32 s_off[kOffWindow + 1];
    __shared__ u32 s_t;
    __shared__ u32 s_stat[3];
    __shared__ u32 s_tbase;
    __shared__ u32 lds8[4];
    for (int i = threadIdx.x; i < VOX; i += 256) { a_w[i] = 0; a_d[i] = 0; a_n[i] = 0; }
    const u32 nt = cs->error ? 0u : cs->t_count * (u32)SPLIT;
    for (;;) {
        if (threadIdx.x == 0) { s_t = atomicAdd(&cs->work_next, 1u); s_stat[0] = 0; s_stat[1] = 0; s_stat[2] = 0; }
        __syncthreads();
        const u32 u = s_t;
        if (u >= nt) break;
        const u32 t = u / (u32)SPLIT;
        const int q = (int)(u % (u32)SPLIT);
        const int lbase = q * VOX;
        const u64 tk = t_key[t];
        const MapDesc& M = maps[(u32)(tk >> 45)];
        if (M.st->error != 0) { __syncthreads(); continue; }
        int bx, by, bz;
        unpack_block(tk & ((1ull << 45) - 1), bx, by, bz);
        const int ts = t_slot[t];
        const bool is_new = (ts & 0x40000000) != 0;
        const size_t slot = (size_t)(ts & 0x3FFFFFFF);
        void* pool = M.pool;
        const size_t vbase = slot * 4096 + (size_t)lbase;
        float D[VPT], W[VPT];
        u32 ntot[VPT];
#pragma unroll
        for (int j = 0; j < VPT; ++j) {
            ntot[j] = 0;
            if (is_new) { D[j] = 0.0f; W[j] = 0.0f; }
            else load_voxel<STORAGE>(pool, vbase + threadIdx.x + 256 * j, D[j], W[j]);
        }
        const int ox = 16 * bx, oy = 16 * by, oz = 16 * bz + q * ZS;
        u32 stat_vox = 0, stat_touch = 0;
        for (int w0 = 0; w0 < M.njobs; w0 += kOffWindow) {
            const int wn = M.njobs - w0 < kOffWindow ? M.njobs - w0 : kOffWindow;
            for (int k = threadIdx.x; k <= wn; k += 256) s_off[k] = off[t * JM + (u32)(w0 + k)];
            __syncthreads();
            // frames of the window in order; the first ray of every thread for the next frame
            // that has rays is loaded while the current frame is processed
            int jm = 0;
            while (jm < wn && s_off[jm] == s_off[jm + 1]) ++jm;
            float4 nxt = make_float4(0.f, 0.f, 0.f, 0.f);
            bool has_nxt = false;
            if (jm < wn) {
                const u32 e = s_off[jm] + threadIdx.x;
                has_nxt = e < s_off[jm + 1];
                if (has_nxt) nxt = sorted[e];
            }
            while (jm < wn) {
                int jn = jm + 1;
                while (jn < wn && s_off[jn] == s_off[jn + 1]) ++jn;
                const float4 cur = nxt;
                const bool has_cur = has_nxt;
                const u32 lo = s_off[jm], hi = s_off[jm + 1];
                if (jn < wn) {
                    const u32 e = s_off[jn] + threadIdx.x;
                    has_nxt = e < s_off[jn + 1];
                    if (has_nxt) nxt = sorted[e];
                }
                const Job& J = jobs[M.job0 + w0 + jm];
                const float s[3] = {J.pose[3], J.pose[7], J.pose[11]};
                for (u32 e = lo + threadIdx.x; e < hi; e += 256) {
                    const float4 rp = e == lo + threadIdx.x ? cur : sorted[e];
                    (void)has_cur;
                    const float p[3] = {rp.x, rp.y, rp.z};
                    float ev[3], r;
                    Walk w;
                    walk_setup(M, p, s, ev, r, w);
                    bool inside = false;
                    for (int guard = 0; guard < kMaxStepsPerRay; ++guard) {
                        const int lx = w.g[0] - ox, ly = w.g[1] - oy, lz = w.g[2] - oz;
                        if ((u32)lx < 16u && (u32)ly < 16u && (u32)lz < (u32)ZS) {
                            inside = true;
                            const Obs o = observe(M, p, ev, r, rp.w, w.g[0], w.g[1], w.g[2]);
                            const u32 l = (u32)lx | ((u32)ly << 4) | ((u32)lz << 8);
                            const u64 fw = (u64)__builtin_rintf(o.w * M.wscale);
                            const i64 fd = (i64)__builtin_rintf(o.w * o.e * M.wscale);
                            if (fw) atomicAdd(&a_w[l], fw);
                            if (fd) atomicAdd(&a_d[l], (u64)fd);
                            atomicAdd(&a_n[l], 1u);
                        } else if (inside) {
                            break;   // the walk is monotone per axis: it never re-enters the slab
                        }
                        if (w.left == 0) break;
                        walk_step(w);
                    }
                }
                __syncthreads();
                // Eqs. (3)-(4), once per voxel for this frame
#pragma unroll
                for (int j = 0; j < VPT; ++j) {
                    const int l = threadIdx.x + 256 * j;
                    const u32 c = a_n[l];
                    if (c) {
                        const u64 sw_fx = a_w[l];
                        if (sw_fx) {
                            const float sw = (float)sw_fx * M.inv_wscale;
                            // sums are in units of delta; binary32 storage keeps D in metres,
                            // binary16 storage keeps D / delta
                            float swd = (float)(i64)a_d[l] * M.inv_wscale;
                            if (STORAGE == 0) swd = swd * M.delta;
                            float Dn = (W[j] * D[j] + swd) / (W[j] + sw);
                            float Wn = W[j] + sw;
                            if (Wn > M.w_max) Wn = M.w_max;
                            if (STORAGE == 1) {
                                Dn = __half2float(__float2half_rn(Dn));
                                Wn = __half2float(__float2half_rn(Wn));
                            }
                            D[j] = Dn;
                            W[j] = Wn;
                        }
                        ntot[j] += c;
                        stat_vox += 1;
                        stat_touch += c;
                        a_w[l] = 0; a_d[l] = 0; a_n[l] = 0;
                    }
                }
                __syncthreads();
                jm = jn;
            }
            __syncthreads();
        }
#pragma unroll
        for (int j = 0; j < VPT; ++j) store_voxel<STORAGE>(pool, vbase + threadIdx.x + 256 * j, D[j], W[j]);
        if (stat_vox) {
            u32 cells = 0;
#pragma unroll
            for (int j = 0; j < VPT; ++j) cells += ntot[j] ? 1u : 0u;
            atomicAdd(&s_stat[0], stat_vox);
            atomicAdd(&s_stat[1], stat_touch);
            atomicAdd(&s_stat[2], cells);
        }
        if (keep_touches) {
            u32 mine = 0;
#pragma unroll
            for (int j = 0; j < VPT; ++j) mine += ntot[j] ? 1u : 0u;
            u32 tot;
            const u32 incl = block_scan_256(mine, lds8, &tot);
            if (threadIdx.x == 0) s_tbase = atomicAdd(&cs->touch_count, tot);
            __syncthreads();
            u32 pos = s_tbase + incl - mine;
#pragma unroll
            for (int j = 0; j < VPT; ++j) {
                if (ntot[j]) {
                    const int l = threadIdx.x + 256 * j;
                    if (pos < touch_cap) {
                        touch_key[pos] = ((u64)(M.map_id) << 57) |
                                         voxel_key_of(ox + (l & 15), oy + ((l >> 4) & 15), oz + (l >> 8));
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

template __global__ void k_update<0, 1>(const Job*, const MapDesc*, const u64*, const int*,
                                         const u32*, const float4*, u32, u64*, u32*, u32, int,
                                         JobStat*, CallState*);
template __global__ void k_update<0, 2>(const Job*, const MapDesc*, const u64*, const int*,
                                         const u32*, const float4*, u32, u64*, u32*, u32, int,
                                         JobStat*, CallState*);
template __global__ void k_update<0, 4>(const Job*, const MapDesc*, const u64*, const int*,
                                         const u32*, const float4*, u32, u64*, u32*, u32, int,
                                         JobStat*, CallState*);
template __global__ void k_update<1, 1>(const Job*, const MapDesc*, const u64*, const int*,
                                         const u32*, const float4*, u32, u64*, u32*, u32, int,
                                         JobStat*, CallState*);
template __global__ void k_update<1, 2>(const Job*, const MapDesc*, const u64*, const int*,
                                         const u32*, const float4*, u32, u64*, u32*, u32, int,
                                         JobStat*, CallState*);
template __global__ void k_update<1, 4>(const Job*, const MapDesc*, const u64*, const int*,
                                         const u32*, const float4*, u32, u64*, u32*, u32, int,
                                         JobStat*, CallState*);

// ---------------------------------------------------------------------------
// finish: commit block counts, fold statistics, clean per-call tables
// ---------------------------------------------------------------------------
// Frees the per-call block set: the listed slots, or the whole table after a failed call
// (whose set may hold keys that never reached the list).
__global__ __launch_bounds__(256) void k_cleanup(u64* __restrict__ tkeys, u32 tkey_cap,
                                                 const u32* __restrict__ tlist, u32 tlist_cap,
                                                 const CallState* __restrict__ cs) {
    const u32 stride = gridDim.x * 256u;
    if (cs->error) {
        for (u32 i = blockIdx.x * 256u + threadIdx.x; i < tkey_cap; i += stride) tkeys[i] = kEmpty;
    } else {
        const u32 nt = cs->t_count < tlist_cap ? cs->t_count : tlist_cap;
        for (u32 i = blockIdx.x * 256u + threadIdx.x; i < nt; i += stride) tkeys[tlist[i]] = kEmpty;
    }
}

__global__ __launch_bounds__(1024) void k_finish(const Job* __restrict__ jobs, int njobs,
                                                 const MapDesc* __restrict__ maps, int nmaps,
                                                 JobStat* __restrict__ jst,
                                                 CallState* __restrict__ cs) {
    if (threadIdx.x == 0) {
        for (int m = 0; m < nmaps; ++m) {
            MapState* st = maps[m].st;
            const bool ok = st->error == 0 && cs->error == 0;
            if (ok) {
                st->new_blocks += st->new_count;
                st->block_count += st->new_count;
                st->calls += 1;
                for (int j = maps[m].job0; j < maps[m].job0 + maps[m].njobs; ++j) {
                    const JobStat& s = jst[j];
                    st->points += jobs[j].n;
                    st->valid += s.valid;
                    st->invalid += s.invalid;
                    st->oob += s.oob_pts + s.oob_rays;
                    st->rays += s.rays - s.oob_rays;
                    st->touches += s.touches;
                    st->voxels += s.voxels;
                    st->cells += s.cells;
                }
            }
            if (cs->error != 0 && st->error == 0) st->error = cs->error;
            st->new_count = 0;
        }
        cs->ray_count = 0;
        cs->cross_count = 0;
        cs->t_count = 0;
        cs->occ_count = 0;
        cs->work_next = 0;
        cs->error = 0;
    }
    __syncthreads();
    for (int j = threadIdx.x; j < njobs; j += blockDim.x) {
        JobStat z;
        z.valid = z.invalid = z.oob_pts = z.oob_rays = z.rays = z.touches = z.voxels = z.cells = 0;
        jst[j] = z;
    }
}

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

}  // namespace vbx
