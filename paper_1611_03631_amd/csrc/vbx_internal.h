// Internal structures and device helpers of the vbx TSDF integrator (gfx950).
//
// Everything here is compiled without floating-point contraction: the traversal,
// validity tests, the sign of the Eq. (1) distance and the grouped-raycasting
// mean are binary32/binary64 operations in a fixed order, so that the voxels a
// ray visits are reproducible bit-for-bit.
#pragma once
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include <cstring>
#include <type_traits>
#include <stdint.h>

#include "vbx_walk.h"

#pragma clang fp contract(off)

namespace vbx {

typedef unsigned long long u64;
typedef long long i64;
typedef unsigned int u32;

constexpr u64 kEmpty = ~0ull;
constexpr int kMergeSpan = 256;    // grouped raycasting: sorted partial groups per merge work chunk
// Grouped raycasting sorts partial groups by (block, frame, eighth of the block's voxels): a
// sort bin then spans at most 4096 / kGroupSubBins distinct voxels.
constexpr int kGroupSubBins = 8;
constexpr u32 kNoRay = 0xFFFFFFFFu;      // job of an empty ray slot
constexpr int kVoxLimit = 1 << 18;     // |voxel index| < 2^18
constexpr int kBlockBias = 1 << 14;    // block indices packed as 15-bit biased fields
constexpr int kTileSimple = 1024;      // points per workgroup, per-point raycasting
constexpr int kTileGroupedW = 32;      // 2-D tile of an organised cloud (grouped)
constexpr int kTileGroupedH = 16;
constexpr int kTileGrouped = kTileGroupedW * kTileGroupedH;  // 512 points
constexpr int kMaxStepsPerRay = 96;    // guard of the traversal check only (walk_setup_vox)

// Per-map parameters and device pointers for one call (copied to the device per call).
struct MapDesc {
    float v, iv, delta, inv_delta;  // voxel size, 1/v (binary32), truncation, 1/delta
    float eps, ramp, w_max, rmax2;  // Eq. (5) epsilon = v, 1/(delta-eps), W_max, max_range^2
    float z_min, wscale, inv_wscale;  // weight fixed-point scale 2^kw and 2^-kw
    float e_max;                    // min(fl(delta * (1/delta)), 1): bound of a clamped d / delta
    int weighting, merge, storage, dist;
    int wbits;                      // grouped-mean weight bits (0: unit weights)
    int njobs, job0;                // this map's frames in the call: jobs [job0, job0+njobs)
    int map_id;
    u64* hkeys;                     // block hash: keys (kEmpty = free)
    int* hslots;                    //             pool slot per key
    u32 hmask;                      // hash capacity - 1
    u32 capacity;                   // pool capacity in blocks
    void* pool;                     // [capacity][4096] float2 (F32: D metres, W) or u32 16-bit pairs (D/delta, W)
    struct MapState* st;
    u32* dirty;                     // [capacity] blocks changed since the ESDF last looked (null: no ESDF)
    int full_ray;                   // 1: rays start at the sensor, else at max(r - delta, 0)
    int max_steps;                  // guard of a ray walk: at least the longest walk's steps
    u32* color;                     // [capacity][4096] packed RGB8 per voxel (null: no colour)
};

// Device-resident counters of a map.
struct MapState {
    u32 block_count;   // committed blocks (pool slots [0, block_count) are in use)
    u32 new_count;     // blocks pending in the current call
    int error;         // sticky vbx_status of the device side
    u32 pad;
    u64 points, valid, invalid, oob, rays, touches, voxels, cells, new_blocks, calls;
};

// One frame of a call.
struct Job {
    const float* pts;
    u32 n, width;     // points; organised row length (0: unorganised)
    u32 map;          // index into the call's MapDesc array
    u32 jm;           // frame index within its map for this call
    u32 tile0;        // first tile of this job in the current launch
    u32 ntiles;
    float pose[12];
    const u32* colors;   // [n] RGBA8 per point (red in the low byte), or null
};

// Counters of one call (device).
struct CallState {
    u32 ray_count;     // ray slots of the call (some may be empty)
    u32 t_count;       // entries of the per-call block set
    u32 work_next;     // persistent work counter of the update kernel
    u32 touch_count;
    int error;         // call-wide error (scratch overflow)
    u32 scan_done;     // workgroups of the current scan that have written their sum
    u32 finish_done;   // workgroups of the call's last kernel that are done
};

// Partial group of one tile (40 bytes): exact integer sums of the tile's points in one voxel.
// The weight sum is below 2^48 (at most 512 points of fixed-point weight at most 2^32), so the
// point count shares its word.
struct Partial {
    u64 so_n;      // sum of fixed-point point weights | (points - 1) << 48
    u64 sq[3];     // n > 1: sums of weight * Q_k (fit 64 bits for a tile of <= 512 points);
                   // n == 1: the point itself and its Q_k, packed by pack_single
    u32 h;         // block-set slot of the voxel's block
    u32 lj;        // local voxel index (12 bits) | frame-in-map index << 12
};
static_assert(sizeof(Partial) == 40, "partial group record");

// Colour sums of a partial group (colour calls, stored at the partial's index): per channel
// the sum of fixed-point point weight * 8-bit channel value.
struct PartialColor {
    u64 sc[3];
};
constexpr u64 kSoMask = (1ull << 48) - 1;
__host__ __device__ inline u64 partial_so_n(u64 so, u32 n) { return so | ((u64)(n - 1u) << 48); }
__host__ __device__ inline u64 partial_so(u64 so_n) { return so_n & kSoMask; }
__host__ __device__ inline u32 partial_n(u64 so_n) { return (u32)(so_n >> 48) + 1u; }

// A one-point partial group carries the point (binary32 world coordinates) and its grid
// fractions Q_k instead of the sums, which follow from them (sum = weight * Q_k).  A group
// that stays a single point casts its ray to exactly that point.
__host__ __device__ inline void pack_single(const float p[3], const u32 Q[3], u64 sq[3]) {
    u32 b[3];
    for (int k = 0; k < 3; ++k) std::memcpy(&b[k], &p[k], 4);
    sq[0] = (u64)b[0] | ((u64)b[1] << 32);
    sq[1] = (u64)b[2] | ((u64)Q[0] << 32);
    sq[2] = (u64)Q[1] | ((u64)Q[2] << 32);
}
__host__ __device__ inline void unpack_single(const u64 sq[3], float p[3], u32 Q[3]) {
    const u32 b[3] = {(u32)sq[0], (u32)(sq[0] >> 32), (u32)sq[1]};
    for (int k = 0; k < 3; ++k) std::memcpy(&p[k], &b[k], 4);
    Q[0] = (u32)(sq[1] >> 32);
    Q[1] = (u32)sq[2];
    Q[2] = (u32)(sq[2] >> 32);
}

__host__ __device__ inline u64 mix64(u64 x) {
    x ^= x >> 33; x *= 0xff51afd7ed558ccdULL;
    x ^= x >> 33; x *= 0xc4ceb9fe1a85ec53ULL;
    x ^= x >> 33;
    return x;
}

__host__ __device__ inline u64 pack_block(int bx, int by, int bz) {
    return ((u64)(u32)(bx + kBlockBias) << 30) | ((u64)(u32)(by + kBlockBias) << 15) |
           (u64)(u32)(bz + kBlockBias);
}
__host__ __device__ inline void unpack_block(u64 k, int& bx, int& by, int& bz) {
    bx = (int)((k >> 30) & 0x7FFF) - kBlockBias;
    by = (int)((k >> 15) & 0x7FFF) - kBlockBias;
    bz = (int)(k & 0x7FFF) - kBlockBias;
}
__host__ __device__ inline u64 block_key_of(int gx, int gy, int gz) {
    return pack_block(gx >> 4, gy >> 4, gz >> 4);   // arithmetic shift = floor division by 16
}
__host__ __device__ inline u32 local_of(int gx, int gy, int gz) {
    return (u32)(gx & 15) | ((u32)(gy & 15) << 4) | ((u32)(gz & 15) << 8);
}
__host__ __device__ inline u64 voxel_key_of(int gx, int gy, int gz) {
    return (block_key_of(gx, gy, gz) << 12) | local_of(gx, gy, gz);
}
__host__ __device__ inline void unpack_voxel(u64 k, int& gx, int& gy, int& gz) {
    int bx, by, bz;
    unpack_block(k >> 12, bx, by, bz);
    gx = 16 * bx + (int)(k & 15);
    gy = 16 * by + (int)((k >> 4) & 15);
    gz = 16 * bz + (int)((k >> 8) & 15);
}

// ---------------------------------------------------------------------------
// 16-bit voxel storage
// ---------------------------------------------------------------------------
// Fixed-point distance code of the VBX_S16 storage: D/delta = i / 32767 with |i| <= 32767,
// the nearest code to the binary32 value (ties to even).  |D/delta| <= 1 always holds for a
// weighted mean of clamped distances; the clamp only absorbs binary32 rounding.
__host__ __device__ inline unsigned short s16_encode(float dn) {
    float x = dn * 32767.0f;
    x = x > 32767.0f ? 32767.0f : (x < -32767.0f ? -32767.0f : x);
    return (unsigned short)(short)(int)__builtin_rintf(x);
}
__host__ __device__ inline float s16_decode(unsigned short c) { return (float)(short)c / 32767.0f; }

// One voxel of a map's pool: D (metres for binary32 storage, D / delta for 16-bit storage)
// and W.
template <int STORAGE>
__device__ inline void load_voxel(const void* pool, size_t idx, float& D, float& W) {
    if (STORAGE == 0) {
        const float2 dw = ((const float2*)pool)[idx];
        D = dw.x; W = dw.y;
    } else {
        // 16-bit pairs: D / delta in the low half (binary16, or the fixed-point code), W
        // (binary16) in the high half
        const u32 raw = ((const u32*)pool)[idx];
        D = STORAGE == 1 ? __half2float(__ushort_as_half((unsigned short)(raw & 0xFFFF)))
                         : s16_decode((unsigned short)(raw & 0xFFFF));
        W = __half2float(__ushort_as_half((unsigned short)(raw >> 16)));
    }
}
// Pool slot of block key bk in the map's hash (linear probing from mix64), -1 if absent.
__device__ inline int find_block(const MapDesc& M, u64 bk) {
    u32 h = (u32)mix64(bk) & M.hmask;
    for (u32 probe = 0; probe <= M.hmask; ++probe) {
        const u64 k = M.hkeys[h];
        if (k == bk) return M.hslots[h];
        if (k == kEmpty) return -1;
        h = (h + 1) & M.hmask;
    }
    return -1;
}

// ---------------------------------------------------------------------------
// Point validity and pose transform (binary32, fixed order)
// ---------------------------------------------------------------------------
// Returns true and the world point q when the sensor-frame point is valid:
// finite, 0 < |p|^2 <= max_range^2, depth z >= z_min under quadratic weighting,
// and the world point's voxel index inside the addressable range.
__device__ inline int classify_point(const MapDesc& M, const float* pose, float x, float y,
                                     float z, float q[3]) {
    // 0 = invalid, 1 = valid, 2 = out of bounds.  Straight-line: every test is evaluated and
    // the class selected at the end.  A non-finite coordinate makes rho2 infinite or NaN, which
    // fails rho2 <= rmax2, so the range test also rejects it.
    const float rho2 = (x * x + y * y) + z * z;
    const bool ok = rho2 > 0.0f && rho2 <= M.rmax2 && (M.weighting != 1 || z >= M.z_min);
    bool inb = true;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        q[k] = ((pose[4 * k] * x + pose[4 * k + 1] * y) + pose[4 * k + 2] * z) + pose[4 * k + 3];
        const float f = q[k] * M.iv;
        inb = inb && f >= -(float)kVoxLimit && f < (float)kVoxLimit;
    }
    return ok ? (inb ? 1 : 2) : 0;
}

// ---------------------------------------------------------------------------
// Ray set-up and traversal of the truncation band (binary32, fixed order)
// ---------------------------------------------------------------------------
// Segment of the ray s->p inside the band [max(r - delta, 0), r + delta]; returns
// false (out of bounds) when r == 0 or an end lies outside the voxel range.
__device__ inline bool walk_setup(const MapDesc& M, const float p[3], const float s[3],
                                  float e[3], float& r, Walk& w) {
#pragma unroll
    for (int k = 0; k < 3; ++k) e[k] = p[k] - s[k];
    r = __builtin_sqrtf((e[0] * e[0] + e[1] * e[1]) + e[2] * e[2]);
    if (r == 0.0f) return false;
    float t0 = M.full_ray ? 0.0f : r - M.delta;
    if (t0 < 0.0f) t0 = 0.0f;
    float t1 = r + M.delta;
    float A[3], B[3];
    bool ok = true;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        float u = e[k] / r;
        float a = s[k] + u * t0;
        float b = s[k] + u * t1;
        A[k] = a * M.iv;
        B[k] = b * M.iv;
        ok = ok && (A[k] >= -(float)kVoxLimit && A[k] < (float)kVoxLimit &&
                    B[k] >= -(float)kVoxLimit && B[k] < (float)kVoxLimit);
    }
    if (!ok) return false;
    w.left = 0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        int ga = (int)__builtin_floorf(A[k]);
        int gb = (int)__builtin_floorf(B[k]);
        w.g[k] = ga;
        w.n[k] = gb > ga ? gb - ga : ga - gb;
        w.step[k] = gb > ga ? 1 : (gb < ga ? -1 : 0);
        w.tM[k] = __builtin_inff();
        w.tD[k] = __builtin_inff();
        if (w.n[k] > 0) {
            float delta = B[k] - A[k];
            float bound = (float)(ga + (w.step[k] > 0 ? 1 : 0));
            w.tD[k] = 1.0f / __builtin_fabsf(delta);
            w.tM[k] = (bound - A[k]) / delta;
        }
        w.left += w.n[k];
    }
    return true;
}

// ---------------------------------------------------------------------------
// Observation of a voxel by a ray: Eq. (1) distance, Eq. (2)/(5) weight
// ---------------------------------------------------------------------------
struct Obs {
    float w;     // weight
    float e;     // clamped distance / delta, in [-1, 1]
};

// DIST: the distance form (M.dist), fixed by the caller for a whole walk.
template <int DIST>
__device__ inline Obs observe(const MapDesc& M, const float p[3], const float e[3], float r,
                              float wgt, int gx, int gy, int gz) {
    // Voxel centre c v, c = g + 1/2 (exact in binary32 for |g| < 2^18).  The rounded product
    // x = fl(c v) decides the sign of Eq. (1) in binary32, in the same operation order on every
    // side.  The distance value is measured from the exact centre instead: the product's
    // remainder c v - x is a binary32 number (an fma gives it exactly), so p - c v is formed
    // with two roundings relative to |p - c v| <= delta + v, not to the world coordinates.
    const float c0 = (float)gx + 0.5f, c1 = (float)gy + 0.5f, c2 = (float)gz + 0.5f;
    const float x0 = c0 * M.v, x1 = c1 * M.v, x2 = c2 * M.v;
    const float f0 = p[0] - x0, f1 = p[1] - x1, f2 = p[2] - x2;
    const float h0 = f0 - __builtin_fmaf(c0, M.v, -x0);
    const float h1 = f1 - __builtin_fmaf(c1, M.v, -x1);
    const float h2 = f2 - __builtin_fmaf(c2, M.v, -x2);
    float d;
    if (DIST == 0) {
        const float dot = (f0 * e[0] + f1 * e[1]) + f2 * e[2];
        // the hardware square root (within 1 ulp of the exact root) of the exact-centre offset
        const float mag = __builtin_amdgcn_sqrtf((h0 * h0 + h1 * h1) + h2 * h2);
        d = dot > 0.0f ? mag : (dot < 0.0f ? -mag : 0.0f);
    } else {
        // the projective distance is continuous in the offset: no binary32 sign decision
        d = ((h0 * e[0] + h1 * e[1]) + h2 * e[2]) / r;
    }
    Obs o;
    float fdrop = 1.0f;
    if (M.weighting == 1) {
        const float ramp = (d + M.delta) * M.ramp;   // selected below, not branched on
        fdrop = d > -M.eps ? 1.0f : (d > -M.delta ? ramp : 0.0f);
    }
    o.w = wgt * fdrop;
    // d clamped to [-delta, delta], over delta, clamped to [-1, 1]: the rounded product is
    // monotone in d and equals e_max at d = delta, so one clamp of d / delta gives the same value
    o.e = __builtin_amdgcn_fmed3f(d * M.inv_delta, -M.e_max, M.e_max);
    return o;
}

// rint(x) (ties to even) as a two's-complement 64-bit integer, for |x| < 2^51: binary64 holds x
// exactly, and adding 1.5 * 2^52 rounds it to an integer, held in the low mantissa bits.
__device__ inline u64 rint_fixed51(float x) {
    const u64 b = (u64)__double_as_longlong((double)x + 6755399441055744.0);
    return ((u64)((u32)(b >> 32) - 0x43380000u) << 32) | (u64)(u32)b;
}

// The fixed-point terms of one observation, rint(w 2^kw) and rint(w e 2^kw).  A wave whose
// weights all lie below 2^51 in fixed point (every ray of fewer than 2^(51 - kw) points'
// weight) takes the short binary64 form; otherwise the general 64-bit conversion.
__device__ inline void fixed_terms(float xw, float xd, u64& fw, u64& fd) {
    fw = rint_fixed51(xw);
    fd = rint_fixed51(xd);
    if (__builtin_expect(__ballot(!(xw < 0x1p51f)) != 0ull, 0)) {   // rare: the general form
        fw = (u64)__builtin_rintf(xw);
        fd = (u64)(i64)__builtin_rintf(xd);
    }
}

}  // namespace vbx
