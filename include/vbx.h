/*
 * vbx — TSDF integration into spatially hashed 16^3-voxel blocks on AMD MI355X
 * (gfx950), after Oleynikova et al., "Voxblox: Incremental 3D Euclidean Signed
 * Distance Fields for On-Board MAV Planning", Sec. III (voxel-hashed layers) and
 * Sec. IV (TSDF construction: Eqs. 1-5, grouped raycasting).
 *
 * C ABI: plain pointers and sizes only.  "dev" pointers are device (HBM) memory
 * of the current HIP device; "host" pointers are ordinary host memory.
 *
 * Conventions
 *  - Every function returns a vbx_status: VBX_OK (0) or a negative error.  Out
 *    parameters are written only on success.  No C++ exception crosses the ABI.
 *  - Integration calls are stream-ordered and asynchronous: they enqueue work on
 *    the map's HIP stream and return.  The caller keeps the point buffers alive
 *    until the stream has passed the call (e.g. vbx_map_sync).
 *  - Errors found on the device (block pool full) are sticky.  The call that hits
 *    them leaves the map exactly as it was before the call; later integration
 *    calls are skipped until vbx_map_reserve (or vbx_map_clear_error) is called.
 *    vbx_map_sync returns the sticky error.
 *  - The map owns its device memory (hash table, block pool, scratch).  Callers
 *    own their input and output buffers.
 *  - Voxel g (integer index, world position (g + 0.5) * voxel_size at its centre)
 *    lives in block floor(g / 16), local index (g - 16*block) with x fastest:
 *    l = lx + 16*ly + 256*lz.
 */
#ifndef VBX_H
#define VBX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    VBX_OK = 0,
    VBX_ERR_INVALID_ARG = -1,      /* bad pointer, size or parameter */
    VBX_ERR_OUT_OF_MEMORY = -2,    /* device or pinned host allocation failed */
    VBX_ERR_POOL_FULL = -3,        /* block pool capacity exceeded; map unchanged by that call */
    VBX_ERR_BUFFER_TOO_SMALL = -4, /* caller's output buffer (or touch record buffer) too small */
    VBX_ERR_DEVICE = -5,           /* a HIP runtime call failed */
    VBX_ERR_LIMIT = -6             /* request beyond a documented limit (points per frame, frames) */
} vbx_status;

/* Weighting of one observation: Eq. (2) constant w = 1, or Eq. (5) 1/z^2 with a
 * linear drop-off behind the surface (epsilon = voxel_size, delta = trunc). */
typedef enum { VBX_W_CONST = 0, VBX_W_QUAD = 1 } vbx_weighting;

/* Raycasting every point, or grouped raycasting (Sec. IV-B): points that fall in
 * one voxel are merged into one ray cast towards their weighted mean. */
typedef enum { VBX_MERGE_NONE = 0, VBX_MERGE_GROUPED = 1 } vbx_merge;

/* Storage of the per-voxel distance D and weight W of Eqs. (3)-(4); the arithmetic is
 * binary32 in every mode, and the stored values are rounded (to nearest, ties to even) once
 * per frame after the update.
 *  VBX_F32: binary32 D (metres) and W, 8 B/voxel.
 *  VBX_F16: binary16 D/trunc and W, 4 B/voxel.  Near |D| = trunc a binary16 D/trunc has
 *           11 significant bits, so each frame's rounding moves D by up to 2^-12 trunc.
 *  VBX_S16: D/trunc as a signed 16-bit fixed-point number (D/trunc = i / 32767, |i| <= 32767)
 *           and W as binary16, 4 B/voxel: the same bytes, with a uniform distance step of
 *           trunc / 32767 everywhere in the band.
 * In both 16-bit modes a frame's update is lost once it is below half a storage step: W stops
 * growing once the frame's summed weight is below half a binary16 ulp of W (W >= 2048 times
 * that weight), and D stops moving once W_sum |d - D| / (W + W_sum) is below half a step. */
typedef enum { VBX_F32 = 0, VBX_F16 = 1, VBX_S16 = 2 } vbx_storage;

/* Distance of Eq. (1) (Euclidean norm with the sign of the projection on the
 * ray) or the projective distance along the ray (Sec. I). */
typedef enum { VBX_DIST_EQ1 = 0, VBX_DIST_ALONG_RAY = 1 } vbx_dist;

enum {
    VBX_FLAG_KEEP_TOUCHES = 1u,  /* record the touched voxels and ray counts of the last call */
    /* Raycasting updates every voxel from the sensor origin to trunc behind the point (the
     * raycasting of Sec. IV-B, which carves the free space in front of the surface), instead of
     * the truncation band [r - trunc, r + trunc] alone.  Needs (max_range + trunc) / voxel_size
     * <= 1024 (VBX_ERR_LIMIT otherwise). */
    VBX_FLAG_FULL_RAY = 2u,
    /* The map keeps a colour per voxel (Sec. IV-B: each grouped ray carries the mean colour of
     * its points), 4 more bytes per voxel.  Raycasting frames of such a map must carry colours
     * (vbx_frame.colors).  Per voxel and frame, with w_i the observation weights of the frame's
     * rays through the voxel and c_i their colours, and W the voxel's weight before the frame:
     *   C <- round((W C + sum w_i c_i) / (W + sum w_i))  per 8-bit channel (nearest, ties even).
     * A grouped ray's colour is round(sum Omega c / sum Omega) over its points (Omega the
     * points' fixed-point weights of the group mean), computed in integers.  Projection mapping
     * leaves colours unchanged.  New voxels and imported blocks start black; blocks that
     * vbx_write_blocks overwrites in place keep their colours.  Calls with a colour map walk one
     * frame per step over block regions (the colour sums need the room of a second frame);
     * results do not depend on it. */
    VBX_FLAG_COLOR = 4u
};

/* Limits */
#define VBX_MAX_POINTS_PER_FRAME (1u << 24)
#define VBX_MAX_FRAMES_PER_CALL 4096
#define VBX_VOXEL_INDEX_LIMIT (1 << 18) /* |voxel index| < 2^18, |block index| < 2^14 */

typedef struct {
    float voxel_size;        /* v, metres, > 0 */
    float trunc;             /* delta, metres, > 0 (the paper uses 4v; 3v is common) */
    float w_max;             /* W_max of Eq. (4); <= 65504 for VBX_F16 and VBX_S16 */
    float max_range;         /* points farther than this from the sensor are rejected */
    float z_min;             /* VBX_W_QUAD: points with depth z < z_min are rejected; >= 0.05 */
    int32_t weighting;       /* vbx_weighting */
    int32_t merge;           /* vbx_merge */
    int32_t storage;         /* vbx_storage */
    int32_t dist;            /* vbx_dist */
    uint32_t block_capacity; /* blocks the pool holds; vbx_map_reserve grows it */
    uint32_t flags;          /* VBX_FLAG_* */
    void* stream;            /* hipStream_t to run on (NULL: the null stream) */
    /* Allocator hook for the map's own device memory: the block hash table, the block pool
     * and the map's device state (a map holds its layer of blocks, Sec. III).  alloc(bytes,
     * alloc_ctx) returns device memory of the current device, aligned to 256 bytes, or NULL
     * when it cannot (the call that needed it then fails with VBX_ERR_OUT_OF_MEMORY and
     * leaves the map as it was); free(ptr, alloc_ctx) returns it.  Both NULL (the default):
     * hipMalloc and hipFree.  Setting only one of them is VBX_ERR_INVALID_ARG.  The hooks are
     * called from the thread that creates, grows or destroys the map, never from a stream.
     * Per-call scratch memory is not the map's storage and always comes from hipMalloc. */
    void* (*alloc)(size_t bytes, void* alloc_ctx);
    void (*free)(void* ptr, void* alloc_ctx);
    void* alloc_ctx;
} vbx_map_params;

/* One depth or LiDAR frame. */
typedef struct {
    const float* points; /* dev [n][3] float32, sensor frame; non-finite marks an invalid point */
    uint64_t n;          /* number of points, <= VBX_MAX_POINTS_PER_FRAME */
    uint32_t width;      /* organised clouds: row length (n % width == 0); 0 = unorganised.
                            Only a locality hint for grouping: results do not depend on it. */
    uint32_t reserved;
    float pose[12];      /* row-major 3x4 T_world_sensor; the sensor origin is its last column */
    const uint32_t* colors; /* dev [n] RGBA8 per point, red in the low byte (alpha unused), for maps
                               with VBX_FLAG_COLOR; NULL otherwise (ignored by other maps) */
} vbx_frame;

typedef struct {
    uint64_t points;        /* points submitted */
    uint64_t valid;         /* points that passed the validity tests */
    uint64_t invalid;       /* non-finite, zero range, beyond max_range, or z < z_min */
    uint64_t out_of_bounds; /* points or ray bands outside the addressable voxel range */
    uint64_t rays;          /* rays cast (points, or groups under VBX_MERGE_GROUPED) */
    uint64_t touches;       /* ray-voxel visits (voxel updates) */
    uint64_t voxels;        /* distinct (voxel, frame) pairs updated */
    uint64_t cells;         /* distinct voxels updated per call, summed over calls */
    uint64_t new_blocks;    /* blocks allocated */
    uint64_t blocks;        /* blocks in the map */
    uint64_t calls;         /* integration calls that ran */
} vbx_stats;

typedef struct vbx_map vbx_map;

/* Fills *p with defaults: w_max 1e4, max_range 5 m, z_min 0.1 m, constant
 * weighting, no grouping, binary32 storage, Eq. (1), capacity 65536 blocks. */
void vbx_default_params(vbx_map_params* p);

/* Creates a map with the defaults above (Sec. III: a layer of blocks indexed by
 * position through a hash table).  voxel_size and trunc in metres; weighting is
 * a vbx_weighting. */
int vbx_map_create(float voxel_size, float trunc, int weighting, vbx_map** out);

/* Creates a map from explicit parameters.  Allocates the hash table (2x the
 * capacity, power of two) and the block pool on the current device. */
int vbx_map_create_ex(const vbx_map_params* params, vbx_map** out);

/* Waits for the map's stream and frees everything the map owns.  NULL is a no-op. */
void vbx_map_destroy(vbx_map* map);

/* Sets the HIP stream later calls run on (hipStream_t, NULL = null stream). */
int vbx_map_set_stream(vbx_map* map, void* stream);

/* Integrates one frame (Sec. IV: raycast every valid point's truncation band,
 * weight each observation by Eq. (2) or (5), merge into each voxel by Eqs. (3)-(4);
 * grouped raycasting per Sec. IV-B when the map merges).  points_dev: dev [n][3]
 * float32 in the sensor frame; pose: host [12] row-major T_world_sensor.
 * All observations of one frame that reach a voxel are merged in one update. */
int vbx_integrate(vbx_map* map, const float* points_dev, size_t n, const float pose[12]);

/* Integrates F frames in order in one pipelined pass (Sec. IV: every frame's observations
 * are merged by Eqs. (3)-(4) in frame order; the frames' rays are independent of the map, so
 * their contributions are computed together and each voxel folds them in order).  The
 * result is bit-identical to F consecutive vbx_integrate calls.  points_dev: host array of F dev pointers;
 * n: host [F]; poses: host [F][12]. */
int vbx_integrate_batch(vbx_map* map, const float* const* points_dev, const size_t* n,
                        const float* poses, int F);

/* As vbx_integrate_batch, with per-frame organisation hints. */
int vbx_integrate_frames(vbx_map* map, const vbx_frame* frames, int F);

/* Integrates F organised depth frames in order by projection mapping (Sec. IV-B) instead of
 * raycasting: every voxel of the blocks the frames' truncation bands cross is projected into the
 * depth image and takes its distance from the depth the image holds there.  frames: host [F],
 * each with width > 0 and n a multiple of it (pixel (i, j) is point i + width j); intrinsics:
 * host [4] = fx, fy, cx, cy, mapping a camera point (x, y, z) to pixel coordinates
 * (fx x / z + cx, fy y / z + cy), pixel (floor(u), floor(v)).  A voxel is observed when its centre
 * lies in front of the camera, projects into the image onto a valid point, and the depth
 * difference d = z_pixel - z_voxel (along the optical axis) exceeds -trunc; it is then updated by
 * Eqs. (3)-(4) with d clamped to +-trunc and the weight of Eq. (2), or of Eq. (5) with the
 * pixel's depth.  One observation per voxel and frame.  The map's merge mode does not apply.
 * INVALID_ARG for unorganised frames or intrinsics that are not finite with fx, fy > 0. */
int vbx_integrate_projective(vbx_map* map, const vbx_frame* frames, int F, const float intrinsics[4]);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid allocation): vbx_integrate_frames into one map, with the call's
 * scratch memory (rays, partial groups, sort bins, block set, tables, counters) taken from a
 * fixed region of VBX_NOALLOC_SCRATCH_BYTES that the library holds on each device it runs on
 * until the process ends.  The call makes no hipMalloc, hipFree or pinned host allocation: the
 * frame and map tables travel in kernel launch arguments, and the region's counters and tables
 * are cleared by fill kernels at the start of every call.  The result is bit-identical to
 * vbx_integrate_frames on the same frames.  Returns VBX_ERR_LIMIT, with nothing launched, when
 * the call needs more scratch than the region holds (one 640x480 frame under grouped raycasting
 * into a map of 65536 blocks needs about 65 MB); VBX_ERR_INVALID_ARG when the map was created on
 * another device than the current one.  Every call on a device shares that device's region and
 * leaves its contents behind: calls that may overlap on one device (different streams without
 * ordering between them) race, so order them on one stream.  Touch records are not kept (a
 * following vbx_last_touches reports VBX_ERR_INVALID_ARG), and stage profiling does not apply. */
#define VBX_NOALLOC_SCRATCH_BYTES ((size_t)128 << 20)
int vbx_integrate_frames_noalloc(vbx_map* map, const vbx_frame* frames, int F);

/* Integrates frames[i] into maps[i] for i < M (distinct maps on one device) in one
 * pipelined pass on maps[0]'s stream, using maps[0]'s scratch memory.  Each map is
 * integrated as in vbx_integrate (Sec. IV); batching independent maps into one pass is this
 * library's own pattern (the paper integrates one map).  Each map's
 * result is bit-identical to integrating its frame alone. */
int vbx_integrate_multi(vbx_map* const* maps, const vbx_frame* frames, int M);

/* ---- captured calls ---------------------------------------------------------------
 * This library's own pattern, not the paper's.  A graph is one integration call (the same work as vbx_integrate_multi, or as
 * vbx_integrate_frames for M = 1) captured once into a HIP graph and replayed with one
 * hipGraphLaunch per call, which removes the per-kernel launch cost of small frames
 * (the many-maps-per-tick pattern).  It is bound to its maps and to the point count and
 * width of every frame; point pointers and poses may change between launches. */
typedef struct vbx_graph vbx_graph;

/* Captures the call that integrates frames[i] into maps[owner[i]] (owner NULL: F == M and
 * frames[i] goes to maps[i]); frames of one map apply in array order.  maps: M distinct
 * maps with equal storage and merge mode; the launches run on maps[0]'s stream.  frames
 * are only inspected here (nothing is integrated).  The graph owns its own scratch memory
 * (the size of one eager call's) and a private capture stream.  Synchronises maps[0]'s
 * stream.  Errors: INVALID_ARG, LIMIT (M > 127, F > VBX_MAX_FRAMES_PER_CALL),
 * OUT_OF_MEMORY, DEVICE; *out is written only on success. */
int vbx_graph_create(vbx_map* const* maps, int M, const vbx_frame* frames, const int* owner, int F,
                     vbx_graph** out);

/* Runs the captured call on maps[0]'s stream (asynchronous, stream-ordered).  frames
 * (host [F], or NULL to reuse the previous launch's) replace the points pointers and
 * poses; every frame must keep the n and width given at capture.  The result is
 * bit-identical to the eager call over the same frames.  The caller keeps the points
 * alive until the stream passes the launch.  Errors: INVALID_ARG (changed shapes, or a
 * map whose storage was reallocated since capture: create a new graph), DEVICE. */
int vbx_graph_launch(vbx_graph* graph, const vbx_frame* frames, int F);

/* Waits for maps[0]'s stream and frees the graph.  NULL is a no-op. */
void vbx_graph_destroy(vbx_graph* graph);

/* Blocks until the map's stream is idle; returns the sticky device error, if any. */
int vbx_map_sync(vbx_map* map);

/* Clears a sticky device error (the map content is unchanged). */
int vbx_map_clear_error(vbx_map* map);

/* Grows the block pool (and hash table) to hold at least block_capacity blocks,
 * keeping every block, and clears a sticky VBX_ERR_POOL_FULL.  Synchronises. */
int vbx_map_reserve(vbx_map* map, uint32_t block_capacity);

/* Number of allocated blocks (synchronises). */
int vbx_map_num_blocks(vbx_map* map, size_t* n_out);

/* Exports the map's layer of blocks (Sec. III: blocks of voxels indexed by their position
 * through a hash table) in ascending (bx, by, bz) order (synchronises).
 * coords: host [cap][3] int32 block indices or NULL; dw: host [cap][4096][2] float32
 * (D in metres, W) or NULL.  With both NULL only *n_out is written.  Returns
 * VBX_ERR_BUFFER_TOO_SMALL if cap is smaller than the block count. */
int vbx_export_blocks(vbx_map* map, int32_t* coords, float* dw, size_t cap, size_t* n_out);

/* Replaces the map content with n blocks (Sec. III layer of blocks; coords host [n][3], dw
 * host [n][4096][2], D in metres) — the inverse of vbx_export_blocks (checkpoint / resume).  Values
 * are rounded to the map's storage type.  Synchronises. */
int vbx_import_blocks(vbx_map* map, const int32_t* coords, const float* dw, size_t n);

/* Exports the voxel colours of a VBX_FLAG_COLOR map (Sec. IV-B), in vbx_export_blocks' block order
 * (synchronises): coords host [cap][3] block indices or NULL; colors host [cap][4096] packed RGB8
 * (red in the low byte, top byte 0; voxel l of a block is (l & 15, (l >> 4) & 15, l >> 8)) or
 * NULL.  VBX_ERR_INVALID_ARG for a map without colour; VBX_ERR_BUFFER_TOO_SMALL as above. */
int vbx_export_colors(vbx_map* map, int32_t* coords, uint32_t* colors, size_t cap, size_t* n_out);

/* Touched voxels of the last integration call (requires VBX_FLAG_KEEP_TOUCHES):
 * coords host [cap][3] voxel indices and counts host [cap] (rays that visited the
 * voxel, summed over the call's frames); unordered.  Synchronises.  NULL buffers:
 * only *n_out is written. */
int vbx_last_touches(vbx_map* map, int32_t* coords, uint32_t* counts, size_t cap, size_t* n_out);

/* Cumulative statistics of the map (synchronises). */
int vbx_map_stats(vbx_map* map, vbx_stats* out);

/* Occupancy of the map's block hash (Sec. III: blocks are indexed by position through a hash
 * table; here open addressing with linear probing from a 64-bit mix of the block key).  slots:
 * table size (twice the pool capacity, rounded up to a power of two, so the pool fills first and
 * there is no separate hash-full status); blocks: keys held; mean_probe / max_probe: slots a
 * lookup of a held block reads, from its home slot to its own (1: found at home).  Synchronises. */
typedef struct {
    uint64_t slots;
    uint64_t blocks;
    double mean_probe;
    uint32_t max_probe;
    uint32_t reserved;
} vbx_hash_stats;
int vbx_map_hash_stats(vbx_map* map, vbx_hash_stats* out);

/* Distance at query points by trilinear interpolation of the map (the accuracy evaluation of
 * Sec. VI-A: ground-truth surface points are looked up in the field, and the interpolated
 * distance is their error).  points_dev: device [n][3] float32, world frame (metres);
 * dist_dev: device [n] float32, written with the distance in metres, or NaN where any of the
 * eight voxels around the point (voxel centres at (i + 1/2) v) is unallocated or unobserved
 * (W = 0) or the point lies outside the voxel index range.  The corner choice and fractions
 * are binary32 (u = x * (1/v) - 1/2, corner floor(u), fraction u - floor(u)); the blend runs
 * along x, then y, then z, in binary32.  Buffers stay owned by the caller and must not overlap.
 * Stream-ordered on the map's stream and asynchronous (the result is ready after a later
 * vbx_map_sync or a stream synchronisation).  n <= VBX_MAX_QUERY_POINTS, else VBX_ERR_LIMIT;
 * VBX_ERR_INVALID_ARG for a NULL map, or NULL buffers with n > 0. */
#define VBX_MAX_QUERY_POINTS (1u << 31)
int vbx_map_interpolate(vbx_map* map, const float* points_dev, size_t n, float* dist_dev);

/* Writes n TSDF blocks into the map (Sec. III layer of blocks): coords host [n][3] block indices,
 * dw host [n][4096][2] (D in metres, W), values rounded to the map's storage.  Blocks the map
 * holds are overwritten in place (same pool slot); missing ones are allocated.  Every written
 * block counts as changed for the next vbx_esdf_update.  VBX_ERR_POOL_FULL (map unchanged) when
 * the new blocks do not fit; VBX_ERR_INVALID_ARG for indices outside the voxel range.
 * Synchronises. */
int vbx_write_blocks(vbx_map* map, const int32_t* coords, const float* dw, size_t n);

/* ---- ESDF layer -----------------------------------------------------------------------
 * The Euclidean signed distance field built from the TSDF (Sec. V-A, Algorithm 1): ESDF voxels
 * co-located with the TSDF voxels.  TSDF voxels with |D| < gamma form the fixed band, which
 * takes its values from the TSDF; the other observed voxels (W > 0) take the distance of the
 * band along 26-neighbour paths (quasi-Euclidean steps v, sqrt(2) v, sqrt(3) v), up to d_max,
 * on their own side of the surface.  Unknown voxels (W = 0) take no distance and pass none on.
 * An update looks at the blocks integration (or vbx_write_blocks / vbx_import_blocks) changed
 * since the last update: voxels whose band value rose, or that left the band, start a raise
 * wave that resets the voxels whose distance came from them; new and changed band voxels and
 * the raise wave's border start a lower wave.  The waves run level by level on the device
 * (each level one launch over its frontier), raise first, then lower; the converged field does
 * not depend on the processing order. */
typedef struct {
    float gamma;       /* fixed band radius (metres, > 0); the paper recommends one voxel */
    float d_max;       /* largest distance the field holds (metres, >= gamma) */
    uint32_t reserved[6];
} vbx_esdf_params;

typedef struct {
    uint64_t updates;          /* vbx_esdf_update calls */
    uint32_t dirty_blocks;     /* blocks looked at by the last update */
    uint32_t raise_rounds;     /* levels of the last update's raise wave */
    uint32_t lower_rounds;     /* levels of the last update's lower wave */
    uint32_t reserved;
    uint64_t voxels;           /* voxels the layer holds (allocated blocks * 4096) */
} vbx_esdf_stats;

/* Attaches an ESDF layer to the map (its memory comes from the map's allocator).  Every block
 * the map holds counts as changed for the first update.  INVALID_ARG for bad parameters or a
 * map that already has a layer. */
int vbx_esdf_enable(vbx_map* map, const vbx_esdf_params* params);

/* Propagates the TSDF changes since the last update into the ESDF layer (Algorithm 1).
 * Synchronises (the host reads the frontier sizes between levels).  Returns the map's sticky
 * error if it has one.  out (may be NULL) receives the layer's statistics. */
int vbx_esdf_update(vbx_map* map, vbx_esdf_stats* out);

/* Exports the ESDF layer block by block in ascending (bx, by, bz) order, the TSDF export's order
 * (synchronises): coords host [cap][3] or NULL; d host [cap][4096] float32 signed distance
 * (metres; 0 for unobserved voxels) or NULL; info host [cap][4096] uint8 or NULL: bit 0
 * observed, bit 1 fixed, bits 2..6 the parent's neighbour index (dx + 1) + 3 (dy + 1) +
 * 9 (dz + 1), 13 for none, bit 7 negative side.  BUFFER_TOO_SMALL when cap is below the
 * block count. */
int vbx_esdf_export(vbx_map* map, int32_t* coords, float* d, uint8_t* info, size_t cap, size_t* n_out);

/* Traversal primitive, for verification: for each i < n, the voxels visited between
 * the voxel-space points A_dev[i] and B_dev[i] (dev [n][3] float32), in order,
 * written to out_dev[i][cap][3] (int32), count to counts_dev[i] (may exceed cap;
 * only cap are written).  Runs on the null stream and synchronises. */
int vbx_debug_traverse(const float* A_dev, const float* B_dev, int n, int32_t* out_dev,
                       int cap, int32_t* counts_dev);

/* The 16^3 blocks of the same traversals, in order, as the integration finds them: from the
 * traversal's block-changing steps alone (Sec. III: a ray is integrated into the blocks its
 * truncation band passes through).  Block indices (voxel index >> 4) to out_dev[i][cap][3]
 * (int32), block count to counts_dev[i] (may exceed cap; -1 for a segment outside the voxel
 * range).  Runs on the null stream and synchronises. */
int vbx_debug_traverse_blocks(const float* A_dev, const float* B_dev, int n, int32_t* out_dev,
                              int cap, int32_t* counts_dev);

/* Removes every block and restarts the statistics (stream-ordered, asynchronous).  The
 * pool keeps its capacity; the next call allocates blocks from the start again. */
int vbx_map_clear(vbx_map* map);

/* Per-stage timing of integration calls.  While enabled, every call records HIP events on
 * the map's stream around each pipeline stage (points, groups, cross, resolve, commit,
 * bins, scan, scatter, update, finish); vbx_map_profile_read synchronises and returns the
 * summed milliseconds and launch counts per stage since the last reset.  "bins" is timed for
 * projection mapping only: raycasting counts its crossings inside the cross stage. */
#define VBX_PROFILE_STAGES 10
typedef struct {
    double ms[VBX_PROFILE_STAGES];
    uint64_t launches[VBX_PROFILE_STAGES];
} vbx_profile;

int vbx_map_profile(vbx_map* map, int enable);
int vbx_map_profile_read(vbx_map* map, vbx_profile* out, int reset);

/* Per-stage timing of only the stages in stage_mask (bit i: stage i; 0 disables timing).
 * Every timed stage adds two event records to the stream, and each record costs the stream
 * a few microseconds, so a caller timing whole calls profiles as few stages as it needs.
 * INVALID_ARG for bits at or above VBX_PROFILE_STAGES. */
int vbx_map_profile_stages(vbx_map* map, uint32_t stage_mask);

/* Name of profile stage i (static string), NULL when out of range. */
const char* vbx_profile_stage_name(int stage);

/* Launch tuning of a map's calls.  Results never depend on it. */
#define VBX_TUNING_CANDIDATES 10
typedef struct {
    int32_t update_split;   /* regions each block is cut into for the update stage (default 1) */
    int32_t update_threads; /* threads per update workgroup (default 1024) */
    int32_t update_columns; /* 0: z-slabs; 1: columns cut across x and y.  The candidates are
                               (split, columns, threads) = (1,0,256) (2,0,256) (4,0,256)
                               (2,1,256) (4,1,256) (8,1,256) (1,0,1024) (2,0,1024) (4,0,1024)
                               (2,0,512) */
    int32_t reserved[5];
} vbx_tuning;

int vbx_map_get_tuning(vbx_map* map, vbx_tuning* out);
int vbx_map_set_tuning(vbx_map* map, const vbx_tuning* tuning);

/* Autotuner: times the integration of frames[0..F) under every candidate tuning on a
 * scratch map with the same parameters (the map itself is not modified), keeps the fastest
 * in the map and writes it to *best (may be NULL).  ms_out (may be NULL, at least
 * VBX_TUNING_CANDIDATES entries) receives each candidate's mean time per call.
 * Synchronises. */
int vbx_map_autotune(vbx_map* map, const vbx_frame* frames, int F, vbx_tuning* best,
                     double* ms_out);

/* ---- map server ---------------------------------------------------------------------
 * This library's own serving pattern (the paper integrates one map on one CPU core); each
 * frame is integrated as in vbx_integrate (Sec. IV).  Many maps (one per robot or sensor) served from one device: integration requests
 * arrive one frame at a time, each for one map; the server batches whatever has arrived
 * into the next call ("tick", the vbx_integrate_multi pass, several frames per map
 * allowed) while the previous tick still runs, so batches form continuously.  Requests
 * of one map are applied in submission order, and a map served in the mix ends
 * bit-identical to the same frames integrated into it alone, in that order.  Every map
 * stays resident in device memory; admission charges each map's storage (hash table and
 * block pool) against a byte budget.  Two host threads run the server: one forms and
 * launches ticks, one waits for them and completes requests. */
typedef struct vbx_server vbx_server;

typedef struct {
    uint64_t budget_bytes;         /* device memory all maps' storage may take (> 0) */
    uint32_t max_frames_per_tick;  /* frames per tick (0: 256; at most VBX_MAX_FRAMES_PER_CALL) */
    uint64_t max_points_per_tick;  /* points per tick (0: 2^24); a larger frame runs alone */
    int32_t max_inflight;          /* ticks queued on the device at once, 1..3 (0: 2) */
    int32_t grow;                  /* nonzero: a map whose pool fills is doubled within the
                                      budget (vbx_map_reserve) and its turned-away requests
                                      run again; zero: they fail with VBX_ERR_POOL_FULL */
    void* stream;                  /* hipStream_t of the ticks; NULL: the server creates a
                                      stream ordered after null-stream work */
} vbx_server_params;

typedef struct {
    uint64_t submitted, completed, failed;   /* requests */
    uint64_t ticks, frames, points, replays; /* frames launched, points completed, requests rerun */
    uint32_t maps, rejected_maps;
    uint64_t budget_bytes, used_bytes;
    double p50_ms, p99_ms, max_ms, mean_ms;  /* arrival -> completion, completed requests */
    double points_per_s;                     /* completed points / (last completion - first arrival) */
    double mean_frames_per_tick;
} vbx_server_summary;

/* Seconds on the server's clock (monotonic); arrival times are given on it. */
double vbx_server_clock(void);

/* Starts a server on the current device.  Errors: INVALID_ARG, OUT_OF_MEMORY, DEVICE. */
int vbx_server_create(const vbx_server_params* params, vbx_server** out);

/* Admits a map (its stream is the server's; params->block_capacity is its initial pool).
 * Returns VBX_ERR_OUT_OF_MEMORY, and counts a rejection, when its storage does not fit in
 * what is left of the budget.  *map_id (0, 1, ...) is written on success. */
int vbx_server_add_map(vbx_server* server, const vbx_map_params* params, int* map_id);

/* Queues one frame for map_id.  frame->points (device) must stay valid and unchanged
 * until the request completes.  t_arrival: vbx_server_clock() time the request arrived
 * (<= 0: now); latency is measured from it.  *ticket (may be NULL) identifies it.
 * Returns at once; errors (INVALID_ARG, LIMIT) mean nothing was queued. */
int vbx_server_submit(vbx_server* server, int map_id, const vbx_frame* frame, double t_arrival,
                      uint64_t* ticket);

/* Blocks until the request completes; writes its status (VBX_OK or the error its map
 * reported) and completion time (server clock). */
int vbx_server_wait(vbx_server* server, uint64_t ticket, int* status, double* t_done);

/* Blocks until every queued request has completed. */
int vbx_server_drain(vbx_server* server);

/* Counters and latency percentiles since the start or the last reset. */
int vbx_server_stats(vbx_server* server, vbx_server_summary* out);

/* Drains, then restarts the counters and latency record (maps keep their contents). */
int vbx_server_reset_stats(vbx_server* server);

/* The map behind map_id (owned by the server; NULL if unknown).  Drain before reading it. */
vbx_map* vbx_server_map(vbx_server* server, int map_id);

/* Drains, stops the threads and frees the server and its maps.  NULL is a no-op. */
void vbx_server_destroy(vbx_server* server);

/* Human-readable name of a status code (static string). */
const char* vbx_status_string(int status);

#ifdef __cplusplus
}
#endif
#endif /* VBX_H */
