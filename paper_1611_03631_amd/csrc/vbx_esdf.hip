// ESDF from the TSDF (Sec. V-A, Algorithm 1) on gfx950: the raise and lower wavefronts of the
// paper's queue algorithm, processed level by level.  Every round is one kernel over the
// current frontier (a list of voxel ids); it writes the next frontier, and a round ends with an
// empty frontier, so every launch exits.
//
// A voxel of the ESDF layer is one 64-bit word, co-located with the TSDF voxel (same pool slot
// and local index):
//   bits 63..32  |d| as binary32 bits (non-negative floats order like their bit patterns)
//   bit  31      negative side of the surface
//   bit  30      observed
//   bit  29      fixed (|d_TSDF| < gamma: the band takes its value from the TSDF)
//   bits  4..0   parent: neighbour index 0..26 of the voxel the distance came from (13: none)
// The lower wave lowers a voxel with one 64-bit atomic minimum on (|d| << 32 | flags | parent):
// the flags of a voxel do not change during the wave, so the minimum orders by distance and
// then by parent index, and the converged field and its parents do not depend on the order in
// which the frontier is processed.
#include "vbx_host.h"

namespace vbx {

namespace {

__device__ inline float esdf_mag(u64 w) { return __uint_as_float((u32)(w >> 32)); }
__device__ inline u64 esdf_word(float mag, u32 low) { return ((u64)__float_as_uint(mag) << 32) | low; }

// Voxel id (slot << 12 | local) of neighbour n (0..26) of voxel (slot, l), or -1 when its block
// is not allocated.
__device__ inline int esdf_neighbour(const EsdfDev& E, u32 slot, u32 l, int n) {
    const int x = (int)(l & 15) + (n % 3 - 1);
    const int y = (int)((l >> 4) & 15) + ((n / 3) % 3 - 1);
    const int z = (int)(l >> 8) + (n / 9 - 1);
    const int bx = x < 0 ? 0 : (x > 15 ? 2 : 1);
    const int by = y < 0 ? 0 : (y > 15 ? 2 : 1);
    const int bz = z < 0 ? 0 : (z > 15 ? 2 : 1);
    const int nb = bx + 3 * by + 9 * bz;
    const int s = nb == 13 ? (int)slot : E.nbr[(size_t)slot * 27 + nb];
    if (s < 0) return -1;
    return (s << 12) | (int)((u32)(x & 15) | ((u32)(y & 15) << 4) | ((u32)(z & 15) << 8));
}

// Appends voxel v to a frontier once per tag: the stamp of v takes the tag, and only the thread
// that changed it appends.  The appending lanes of a wave reserve their positions with one
// atomic (a frontier counter is shared by the whole grid, and single-address atomics are
// carried out one after another).
__device__ inline void esdf_push(u32* list, u32* count, u32* stamp, u32 tag, u32 v, u32 cap) {
    const bool app = atomicExch(&stamp[v], tag) != tag;
    const u64 m = __ballot(app);                        // over the lanes that reached this call
    if (m == 0ull) return;
    const int lane = __lane_id();
    const int leader = __ffsll((long long)m) - 1;
    u32 base = 0;
    if (lane == leader) base = atomicAdd(count, (u32)__popcll(m));
    base = (u32)__shfl((int)base, leader);
    if (app) {
        const u32 i = base + (u32)__popcll(m & ((1ull << lane) - 1ull));
        if (i < cap) list[i] = v;
    }
}

}  // namespace

// Slot -> block key, from the map's hash table.
__global__ void k_esdf_slot_keys(const u64* __restrict__ hkeys, const int* __restrict__ hslots, u32 hcap,
                                 u64* __restrict__ slot_key) {
    for (u32 i = blockIdx.x * blockDim.x + threadIdx.x; i < hcap; i += gridDim.x * blockDim.x) {
        const u64 k = hkeys[i];
        if (k != kEmpty) slot_key[hslots[i]] = k;
    }
}

// The 27 neighbour blocks' slots (-1: not allocated) of every committed block.
__global__ void k_esdf_neighbours(const MapDesc M, const u64* __restrict__ slot_key, u32 nblocks,
                                  int* __restrict__ nbr) {
    for (u32 i = blockIdx.x * blockDim.x + threadIdx.x; i < nblocks * 27u; i += gridDim.x * blockDim.x) {
        const u32 slot = i / 27u;
        const int n = (int)(i % 27u);
        int bx, by, bz;
        unpack_block(slot_key[slot], bx, by, bz);
        bx += n % 3 - 1;
        by += (n / 3) % 3 - 1;
        bz += n / 9 - 1;
        const int lim = kVoxLimit / 16;
        int s = -1;
        if (bx >= -lim && bx < lim && by >= -lim && by < lim && bz >= -lim && bz < lim)
            s = n == 13 ? (int)slot : find_block(M, pack_block(bx, by, bz));
        nbr[i] = s;
    }
}

// Blocks whose TSDF changed since the last update (flags set by the integration), listed and
// cleared.
__global__ void k_esdf_dirty_list(u32* __restrict__ dirty, u32 nblocks, u32* __restrict__ list,
                                  u32* __restrict__ count) {
    for (u32 s = blockIdx.x * blockDim.x + threadIdx.x; s < nblocks; s += gridDim.x * blockDim.x) {
        if (dirty[s]) {
            dirty[s] = 0;
            list[atomicAdd(count, 1u)] = s;
        }
    }
}

// Algorithm 1, the loop over updated TSDF voxels: every voxel of every dirty block is compared
// with its ESDF voxel.  A voxel whose TSDF state the ESDF already holds (the same band value, or
// an observed voxel outside the band on the same side) is left, which the listing does too for
// unchanged input; the other cases follow the listing with the readings of the oracle.
template <int STORAGE>
__global__ void k_esdf_seed(const MapDesc M, EsdfDev E, u32 tag_raise, u32 tag_lower) {
    const u32 nd = E.cnt[kEsdfDirtyCount];
    for (u32 i = blockIdx.x * blockDim.x + threadIdx.x; i < nd * 4096u; i += gridDim.x * blockDim.x) {
        const u32 slot = E.list[i >> 12], l = i & 4095u;
        const u32 v = (slot << 12) | l;
        float D, W;
        load_voxel<STORAGE>(M.pool, (size_t)slot * 4096 + l, D, W);
        if (!(W > 0.0f)) continue;                         // unknown voxel: not updated
        const float dT = STORAGE == 0 ? D : D * M.delta;
        const u64 w = E.vox[v];
        const u32 low = (u32)w;
        const bool observed = (low & kEsdfObserved) != 0, was_fixed = (low & kEsdfFixed) != 0;
        const u32 side = dT < 0.0f ? kEsdfNeg : 0u;
        if (-E.gamma < dT && dT < E.gamma) {
            const float old = (low & kEsdfNeg) ? -esdf_mag(w) : esdf_mag(w);
            if (observed && was_fixed && old == dT) continue;      // the band value it holds
            E.vox[v] = esdf_word(__builtin_fabsf(dT), side | kEsdfObserved | kEsdfFixed | kEsdfNoParent);
            if (observed) esdf_push(E.raise[0], &E.cnt[kEsdfRaiseCount], E.rstamp, tag_raise, v, E.fcap);
            esdf_push(E.lower[0], &E.cnt[kEsdfLowerCount], E.lstamp, tag_lower, v, E.fcap);
        } else if (was_fixed || (observed && side != (low & kEsdfNeg))) {
            // left the band, or changed side outside it: back to d_max on its (new) side, and
            // the voxels that took their distance from it are raised
            E.vox[v] = esdf_word(E.d_max, side | kEsdfObserved | kEsdfNoParent);
            esdf_push(E.raise[0], &E.cnt[kEsdfRaiseCount], E.rstamp, tag_raise, v, E.fcap);
        } else if (!observed) {
            // a new voxel outside the band: d_max on its side; its neighbours pass it distances.
            // Only a neighbour that holds a distance below d_max (or is fixed) can pass one: a
            // neighbour at d_max, or unobserved, offers nothing; one that changes in this update
            // enters the waves through its own seed.
            E.vox[v] = esdf_word(E.d_max, side | kEsdfObserved | kEsdfNoParent);
            for (int n = 0; n < 27; ++n) {
                if (n == 13) continue;
                const int u = esdf_neighbour(E, slot, l, n);
                if (u < 0) continue;
                const u64 wu = E.vox[u];
                const u32 lu = (u32)wu;
                if (!(lu & kEsdfObserved)) continue;
                if (!(lu & kEsdfFixed) && !(esdf_mag(wu) < E.d_max)) continue;
                esdf_push(E.lower[0], &E.cnt[kEsdfLowerCount], E.lstamp, tag_lower, (u32)u, E.fcap);
            }
        }
    }
}

// One raise round: every voxel of the frontier that is not fixed returns to d_max on its side
// and loses its parent; each observed neighbour whose parent is this voxel is raised next round,
// every other observed neighbour joins the lower wave's first frontier.  Counters rotate over
// three words: this round reads cnt[r % 3], appends to cnt[(r + 1) % 3] and clears the one the
// next round appends to.
//
// A small frontier is spread over more lanes: each frontier voxel gets L lanes (L a power of
// two up to 32, as many as let the grid take every voxel at once), lane j of a voxel handling
// neighbours j, j + L, ... .  A round then waits for about 27 / L neighbour loads in a row
// rather than 26; a large frontier keeps one lane per voxel, as the grid is full anyway.
__device__ inline u32 esdf_lanes(u64 nv) {
    const u64 T = (u64)gridDim.x * blockDim.x;
    u32 L = 32;
    while (L > 1 && nv * L > T) L >>= 1;
    return L;
}

__global__ void k_esdf_raise(EsdfDev E, u32 r, u32 tag_next, u32 tag_lower) {
    const u32 n_in = E.cnt[kEsdfRaiseCount + r % 3];
    if (blockIdx.x == 0 && threadIdx.x == 0) E.cnt[kEsdfRaiseCount + (r + 2) % 3] = 0;
    if (n_in == 0) return;
    const u32* in = E.raise[r & 1];
    u32* out = E.raise[(r + 1) & 1];
    u32* n_out = &E.cnt[kEsdfRaiseCount + (r + 1) % 3];
    const u64 nv = n_in < E.fcap ? n_in : E.fcap;
    const u32 L = esdf_lanes(nv);
    for (u64 i = (u64)blockIdx.x * blockDim.x + threadIdx.x; i < nv * L; i += (u64)gridDim.x * blockDim.x) {
        const u32 v = in[i / L];
        const u32 slot = v >> 12, l = v & 4095u;
        for (int n = (int)(i % L); n < 27; n += (int)L) {
            if (n == 13) {   // the voxel itself: its reset
                const u32 low = (u32)E.vox[v];
                if (!(low & kEsdfFixed)) E.vox[v] = esdf_word(E.d_max, (low & ~kEsdfParentMask) | kEsdfNoParent);
                continue;
            }
            const int u = esdf_neighbour(E, slot, l, n);
            if (u < 0) continue;
            const u64 wu = E.vox[u];
            const u32 lu = (u32)wu;
            if (!(lu & kEsdfObserved)) continue;
            if (!(lu & kEsdfFixed) && (lu & kEsdfParentMask) == (u32)(26 - n))
                esdf_push(out, n_out, E.rstamp, tag_next, (u32)u, E.fcap);
            else if ((lu & kEsdfFixed) || esdf_mag(wu) < E.d_max)   // one at d_max offers nothing
                esdf_push(E.lower[0], &E.cnt[kEsdfLowerCount], E.lstamp, tag_lower, (u32)u, E.fcap);
        }
    }
}

// One lower round: every observed voxel of the frontier offers each observed neighbour that is
// not fixed its distance plus the step (on the neighbour's side; distances cross the surface
// only from fixed voxels, and a candidate stops at zero).  A neighbour it brings closer to the
// surface joins the next frontier.  Buffers alternate and counters rotate as in the raise.
__global__ void k_esdf_lower(EsdfDev E, u32 r, u32 tag_next) {
    const u32 n_in = E.cnt[kEsdfLowerCount + r % 3];
    if (blockIdx.x == 0 && threadIdx.x == 0) E.cnt[kEsdfLowerCount + (r + 2) % 3] = 0;
    if (n_in == 0) return;
    const u32* in = E.lower[r & 1];
    u32* out = E.lower[(r + 1) & 1];
    u32* n_out = &E.cnt[kEsdfLowerCount + (r + 1) % 3];
    const u64 nv = n_in < E.fcap ? n_in : E.fcap;
    const u32 L = esdf_lanes(nv);   // lanes per frontier voxel, as in the raise
    for (u64 i = (u64)blockIdx.x * blockDim.x + threadIdx.x; i < nv * L; i += (u64)gridDim.x * blockDim.x) {
        const u32 v = in[i / L];
        const u32 slot = v >> 12, l = v & 4095u;
        const u64 wv = E.vox[v];
        const u32 lv = (u32)wv;
        if (!(lv & kEsdfObserved)) continue;
        const float dv = (lv & kEsdfNeg) ? -esdf_mag(wv) : esdf_mag(wv);
        const bool vfixed = (lv & kEsdfFixed) != 0;
        for (int n = (int)(i % L); n < 27; n += (int)L) {
            if (n == 13) continue;
            const int u = esdf_neighbour(E, slot, l, n);
            if (u < 0) continue;
            const u64 wu = E.vox[u];
            const u32 lu = (u32)wu;
            if (!(lu & kEsdfObserved) || (lu & kEsdfFixed)) continue;
            if (!vfixed && ((lu ^ lv) & kEsdfNeg)) continue;
            const int k2 = (n % 3 != 1) + ((n / 3) % 3 != 1) + (n / 9 != 1);   // squared offset length
            const float dist = E.step[k2];
            float c;
            if (lu & kEsdfNeg) {
                c = dv - dist;
                c = c > 0.0f ? 0.0f : c;
            } else {
                c = dv + dist;
                c = c < 0.0f ? 0.0f : c;
            }
            const float mag = __builtin_fabsf(c);
            const u64 key = esdf_word(mag, (lu & ~kEsdfParentMask) | (u32)(26 - n));
            if (key < wu) {
                const u64 old = atomicMin((unsigned long long*)&E.vox[u], (unsigned long long)key);
                if ((u32)(old >> 32) > __float_as_uint(mag)) esdf_push(out, n_out, E.lstamp, tag_next, (u32)u, E.fcap);
            }
        }
    }
}

template __global__ void k_esdf_seed<0>(const MapDesc, EsdfDev, u32, u32);
template __global__ void k_esdf_seed<1>(const MapDesc, EsdfDev, u32, u32);
template __global__ void k_esdf_seed<2>(const MapDesc, EsdfDev, u32, u32);

}  // namespace vbx
