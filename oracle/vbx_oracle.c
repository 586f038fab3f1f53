/*
 * CPU oracle for TSDF integration into hashed 16^3-voxel blocks
 * (Oleynikova et al., "Voxblox", Sec. IV "TSDF Construction").
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library may include, link,
 * load or call this file: only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark use it.  It shares no code, header, table or
 * constant generator with the GPU path.
 *
 * It is deliberately plain and slow: one thread, a simple hash map, every step
 * written in the order the paper describes it.
 *
 * Two tiers of arithmetic:
 *  - Geometry (which voxels a ray visits, which blocks exist, how many rays
 *    touch a voxel, the sign of the Eq. (1) distance, the point validity tests
 *    and the grouped-raycasting mean used to cast the group's ray) is decided in
 *    IEEE binary32, round-to-nearest-even, no fused multiply-add, in the exact
 *    operation order written below.  These are the decisions the GPU kernel
 *    takes too, so both sides must take them in the same precision.
 *  - Values (the distances d, weights w, and the running D, W of Eqs. (3)-(4))
 *    are computed in binary64.  The point p of Eq. (1) is the ray's end point
 *    as the geometry tier fixes it (the binary32 world point, or the binary32
 *    end point of a group's ray), promoted exactly: the voxels a ray visits and
 *    the distances it reports are measured from one and the same point.  The
 *    voxel centre is (g + 1/2) v with v the binary32 voxel size, exact in
 *    binary64.  With world64 set, p is instead the binary64 transform of the
 *    sensor point (and a group's exact binary64 weighted mean): that mode
 *    measures how far binary32 world coordinates move the field.
 *
 * Build: gcc -O2 -std=c11 -ffp-contract=off -fno-fast-math (x86-64 SSE: every
 * float operation is rounded to binary32).
 *
 * Readings of the paper used here (the paper does not fix these details):
 *  - Eq. (1) is used literally: Euclidean norm of p - x with the sign of
 *    (p - x).(p - s), sign(0) = 0.  A flag selects the projective distance
 *    along the ray instead.
 *  - Raycasting updates the truncation band only: the segment of the ray from
 *    max(r - delta, 0) to r + delta, r = |p - s|.  With full_ray set it updates the
 *    whole ray, from the sensor origin to delta behind the point (the raycasting of
 *    Sec. IV-B: "from the center to truncation distance delta behind the point").
 *  - Ray traversal is the Amanatides-Woo grid walk with a fixed step count;
 *    when two axes cross a voxel face at the same parameter the lowest axis
 *    (x, then y, then z) steps first.
 *  - Voxel g has centre (g + 0.5) v; block = floor(g / 16); local = g - 16 block.
 *  - Constant weighting (Eq. 2) is w = 1 with no drop-off.  Quadratic weighting
 *    (Eq. 5) uses z = the point's depth in the sensor frame, epsilon = v and
 *    delta = the map's truncation distance.
 *  - The distance merged into D is clamped to [-delta, delta]; the weight uses
 *    the unclamped distance.
 *  - Eqs. (3)-(4) are applied once per voxel per frame with the summed weight
 *    and weighted distance of all of the frame's rays through that voxel.
 *  - Grouped raycasting: points are grouped by the voxel that contains them;
 *    the group's ray is cast once towards the weighted mean of its points (weights
 *    1 or 1/z^2) and carries the summed weight of the group.  A voxel's
 *    observation count counts rays (groups), not points.
 *  - New blocks start at D = 0, W = 0 (unknown).  A voxel visited by a ray
 *    allocates its block even when the weight it receives is 0.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ */
/* Public structures (mirrored by the Python ctypes wrapper)           */
/* ------------------------------------------------------------------ */
typedef struct {
    float voxel_size;  /* v */
    float trunc;       /* delta */
    float w_max;       /* W_max of Eq. (4); +inf for no cap */
    float max_range;   /* maximum sensor ray length */
    float z_min;       /* quadratic weighting: smallest accepted depth */
    int weighting;     /* 0: Eq. (2) constant; 1: Eq. (5) quadratic with drop-off */
    int merge;         /* 0: raycast every point; 1: grouped raycasting */
    int fp16;          /* 1: round D/delta and W to binary16 after every frame;
                          2: round D/delta to the nearest multiple of 1/32767 (ties to even)
                          and W to binary16 after every frame (16-bit fixed-point distance) */
    int dist;          /* 0: Eq. (1); 1: projective distance along the ray */
    int world64;       /* 1: distances from the binary64 world point (see the header) */
    int full_ray;      /* 1: a ray updates every voxel from the sensor to delta behind its point */
    int color;         /* 1: points carry colours; each voxel keeps the weighted mean colour */
} orc_params;

typedef struct {
    uint64_t points, valid, invalid, out_of_bounds, rays, touches, voxels, new_blocks;
} orc_stats;

#define ORC_VOX_LIMIT 262144 /* |voxel index| < 2^18, i.e. |block index| < 2^14 */

/* ------------------------------------------------------------------ */
/* A plain open-addressing hash map from packed integer keys            */
/* ------------------------------------------------------------------ */
typedef struct {
    double D, W, mass;      /* running distance (in units of delta), weight, sum of ray weights */
    double ramp;            /* sum of the weights of rays seen on the Eq. (5) ramp (-delta < d <= -eps):
                               a diagnostic for comparisons, never part of D or W */
    double sw, swd;         /* this frame's sums */
    double C[3];            /* colour (0..255 per channel, an integer after every frame) */
    double swc[3];          /* this frame's sums of weight * ray colour */
    uint32_t n;             /* this frame's ray count */
    uint32_t stamp;         /* frame in which sw, swd, n were last reset */
} orc_voxel;

typedef struct {
    uint64_t* keys;   /* key + 1; 0 = empty */
    void* vals;
    size_t cap, size, vsize;
} orc_table;

static uint64_t mix64(uint64_t x) {
    x ^= x >> 33; x *= 0xff51afd7ed558ccdULL;
    x ^= x >> 33; x *= 0xc4ceb9fe1a85ec53ULL;
    x ^= x >> 33;
    return x;
}

static void table_init(orc_table* t, size_t vsize) {
    t->cap = 1024; t->size = 0; t->vsize = vsize;
    t->keys = (uint64_t*)calloc(t->cap, sizeof(uint64_t));
    t->vals = calloc(t->cap, vsize);
}

static void table_free(orc_table* t) { free(t->keys); free(t->vals); t->keys = NULL; t->vals = NULL; }

static void* table_get(orc_table* t, uint64_t key, int create, int* created);

static void table_grow(orc_table* t) {
    orc_table n;
    n.cap = t->cap * 2; n.size = 0; n.vsize = t->vsize;
    n.keys = (uint64_t*)calloc(n.cap, sizeof(uint64_t));
    n.vals = calloc(n.cap, n.vsize);
    for (size_t i = 0; i < t->cap; ++i) {
        if (!t->keys[i]) continue;
        int c;
        void* v = table_get(&n, t->keys[i] - 1, 1, &c);
        memcpy(v, (char*)t->vals + i * t->vsize, t->vsize);
    }
    table_free(t);
    *t = n;
}

static void* table_get(orc_table* t, uint64_t key, int create, int* created) {
    if (created) *created = 0;
    if (create && 2 * (t->size + 1) > t->cap) table_grow(t);
    size_t mask = t->cap - 1, i = (size_t)mix64(key) & mask;
    for (;;) {
        if (t->keys[i] == key + 1) return (char*)t->vals + i * t->vsize;
        if (t->keys[i] == 0) {
            if (!create) return NULL;
            t->keys[i] = key + 1;
            memset((char*)t->vals + i * t->vsize, 0, t->vsize);
            t->size++;
            if (created) *created = 1;
            return (char*)t->vals + i * t->vsize;
        }
        i = (i + 1) & mask;
    }
}

/* Voxel and block coordinates are packed with a bias so that keys are non-negative. */
static uint64_t pack3(int32_t a, int32_t b, int32_t c) {
    return ((uint64_t)(uint32_t)(a + (1 << 20)) << 42) | ((uint64_t)(uint32_t)(b + (1 << 20)) << 21) |
           (uint64_t)(uint32_t)(c + (1 << 20));
}
static void unpack3(uint64_t k, int32_t* a, int32_t* b, int32_t* c) {
    *a = (int32_t)((k >> 42) & 0x1FFFFF) - (1 << 20);
    *b = (int32_t)((k >> 21) & 0x1FFFFF) - (1 << 20);
    *c = (int32_t)(k & 0x1FFFFF) - (1 << 20);
}

/* floor(g / 16) for any sign of g */
static int32_t block_of(int32_t g) { return g >= 0 ? g / 16 : -((-g + 15) / 16); }

/* ------------------------------------------------------------------ */
/* The map                                                             */
/* ------------------------------------------------------------------ */
typedef struct {
    orc_params P;
    orc_table vox;      /* voxel key -> orc_voxel */
    orc_table blocks;   /* block key -> (unused byte) */
    uint32_t frame;     /* frames integrated so far */
    /* touches of the last frame */
    uint64_t* touch_keys;
    uint32_t* touch_n;
    size_t n_touch, touch_cap;
    orc_stats last;
} orc_map;

orc_map* orc_create(const orc_params* p) {
    orc_map* m = (orc_map*)calloc(1, sizeof(orc_map));
    m->P = *p;
    table_init(&m->vox, sizeof(orc_voxel));
    table_init(&m->blocks, 1);
    return m;
}

void orc_destroy(orc_map* m) {
    if (!m) return;
    table_free(&m->vox);
    table_free(&m->blocks);
    free(m->touch_keys);
    free(m->touch_n);
    free(m);
}

/* ------------------------------------------------------------------ */
/* Binary16 rounding (round to nearest even, finite saturation at 65504) */
/* ------------------------------------------------------------------ */
double orc_round_half(double x) {
    if (x == 0.0 || !isfinite(x)) return x;
    double ax = fabs(x);
    int e;
    frexp(ax, &e);                 /* ax = m 2^e, m in [0.5, 1) */
    int q = e - 11;                /* 11 significant bits */
    if (q < -24) q = -24;          /* subnormal spacing 2^-24 */
    double ulp = ldexp(1.0, q);
    double r = nearbyint(ax / ulp) * ulp;
    if (r > 65504.0) r = 65504.0;
    return copysign(r, x);
}

/* Fixed-point distance storage: D/delta as i / 32767 with |i| <= 32767, i the nearest integer
   to 32767 D/delta (ties to even). */
double orc_round_s16(double x) {
    double i = nearbyint(x * 32767.0);
    if (i > 32767.0) i = 32767.0;
    if (i < -32767.0) i = -32767.0;
    return i / 32767.0;
}

/* ------------------------------------------------------------------ */
/* Grid traversal (binary32)                                           */
/* ------------------------------------------------------------------ */
/*
 * Visits the voxels of the segment from A to B (coordinates in voxel units,
 * i.e. already multiplied by 1/v).  Writes at most cap voxels to out[3*i..]
 * in visiting order and returns the number visited (sum of the per-axis index
 * differences plus one).
 */
int orc_dda(const float A[3], const float B[3], int32_t* out, int cap) {
    int32_t g[3], n[3], step[3];
    float tM[3], tD[3];
    int total = 0;
    for (int k = 0; k < 3; ++k) {
        int32_t ga = (int32_t)floorf(A[k]);
        int32_t gb = (int32_t)floorf(B[k]);
        g[k] = ga;
        n[k] = gb > ga ? gb - ga : ga - gb;
        step[k] = gb > ga ? 1 : (gb < ga ? -1 : 0);
        tM[k] = INFINITY;
        tD[k] = INFINITY;
        if (n[k] > 0) {
            float delta = B[k] - A[k];
            float bound = (float)(ga + (step[k] > 0 ? 1 : 0));
            tD[k] = 1.0f / fabsf(delta);
            tM[k] = (bound - A[k]) / delta;
        }
        total += n[k];
    }
    int count = 0;
    if (count < cap) { out[0] = g[0]; out[1] = g[1]; out[2] = g[2]; }
    count++;
    for (int s = 0; s < total; ++s) {
        /* among axes with steps left, the smallest crossing parameter; ties -> lowest axis */
        int axis = -1;
        for (int k = 0; k < 3; ++k) {
            if (n[k] == 0) continue;
            if (axis < 0 || tM[k] < tM[axis]) axis = k;
        }
        g[axis] += step[axis];
        n[axis] -= 1;
        tM[axis] = tM[axis] + tD[axis];
        if (count < cap) { out[3 * count] = g[0]; out[3 * count + 1] = g[1]; out[3 * count + 2] = g[2]; }
        count++;
    }
    return count;
}

/* ------------------------------------------------------------------ */
/* Rays                                                                */
/* ------------------------------------------------------------------ */
typedef struct {
    float p32[3];     /* ray end point used for traversal and the sign of Eq. (1) */
    double p64[3];    /* ray end point used for distance values (binary64) */
    double wgt;       /* 1 or 1/z^2 for a point; the summed point weights for a group */
    double col[3];    /* the point's colour, or the group's weighted mean colour (integers) */
} orc_ray;

static int weight_scale_bits(const orc_params* P) {
    /* grouped mean: point weights are fixed-point numbers with 32 - c fractional bits,
       where 2^c is the smallest power of two >= the largest possible weight 1/z_min^2 */
    if (P->weighting == 0) return 0;
    float wmax = 1.0f / (P->z_min * P->z_min);
    int c = 0;
    while (ldexpf(1.0f, c) < wmax) ++c;
    return 32 - c;
}

/* A point's integer weight in a group's exact means: Omega = rint(w 2^s), or 1 under constant
   weighting. */
static uint64_t group_weight(int wbits, float w) {
    return wbits > 0 ? (uint64_t)rintf(ldexpf(w, wbits)) : 1u;
}

/*
 * The ray end point of a group of points (grouped raycasting).  The weighted mean
 * is taken in exact integer arithmetic so that it does not depend on the order
 * in which points are summed:
 *   key_k = floor(f_k) with f_k = p_k * (1/v);  q_k = f_k - key_k (binary32),
 *   Q_k = min(rint(q_k 2^20), 2^20 - 1),  Omega = rint(w 2^s) (s = weight_scale_bits, Omega = 1
 *   for constant weighting),  m_k = (sum Omega Q_k) / (2^20 sum Omega)  (binary64, the 128-bit
 *   integer numerator converted as hi 2^64 + lo),  mean_k = (key_k + m_k) v  rounded to binary32.
 * A group of a single point keeps the point itself.
 */
void orc_group_mean(const float* p32, const float* w32, int n, float v, int wbits, float out[3]) {
    if (n == 1) { out[0] = p32[0]; out[1] = p32[1]; out[2] = p32[2]; return; }
    const float iv = 1.0f / v;
    int32_t key[3];
    for (int k = 0; k < 3; ++k) key[k] = (int32_t)floorf(p32[k] * iv);
    uint64_t so = 0;
    unsigned __int128 sq[3] = {0, 0, 0};
    for (int i = 0; i < n; ++i) {
        uint64_t om = group_weight(wbits, w32[i]);
        so += om;
        for (int k = 0; k < 3; ++k) {
            float f = p32[3 * i + k] * iv;
            float q = f - (float)key[k];
            float qs = rintf(ldexpf(q, 20));
            uint64_t Q = (uint64_t)qs;
            if (Q > (1u << 20) - 1) Q = (1u << 20) - 1;
            sq[k] += (unsigned __int128)om * Q;
        }
    }
    for (int k = 0; k < 3; ++k) {
        double hi = (double)(uint64_t)(sq[k] >> 64);
        double lo = (double)(uint64_t)sq[k];
        double num = hi * 18446744073709551616.0 + lo;
        double den = (double)so * 1048576.0;
        double m = num / den;
        out[k] = (float)(((double)key[k] + m) * (double)v);
    }
}

/* ------------------------------------------------------------------ */
/* Integration of one frame                                            */
/* ------------------------------------------------------------------ */
typedef struct { uint64_t key; uint32_t idx; } orc_keyidx;

static int cmp_keyidx(const void* a, const void* b) {
    const orc_keyidx* x = (const orc_keyidx*)a;
    const orc_keyidx* y = (const orc_keyidx*)b;
    if (x->key != y->key) return x->key < y->key ? -1 : 1;
    return x->idx < y->idx ? -1 : (x->idx > y->idx);
}

static void add_touch(orc_map* m, uint64_t key) {
    if (m->n_touch == m->touch_cap) {
        m->touch_cap = m->touch_cap ? 2 * m->touch_cap : 4096;
        m->touch_keys = (uint64_t*)realloc(m->touch_keys, m->touch_cap * sizeof(uint64_t));
        m->touch_n = (uint32_t*)realloc(m->touch_n, m->touch_cap * sizeof(uint32_t));
    }
    m->touch_keys[m->n_touch++] = key;
}

/* Eq. (5) drop-off factor (1 in front of -epsilon, linear to 0 at -delta, 0 behind) */
static double dropoff(double d, double eps, double delta) {
    if (d > -eps) return 1.0;
    if (d > -delta) return (d + delta) / (delta - eps);
    return 0.0;
}

/* G2: the world point of a sensor point (binary32, fixed order). */
static void transform_point(const float pose[12], float x, float y, float z, float q[3]) {
    for (int k = 0; k < 3; ++k)
        q[k] = ((pose[4 * k] * x + pose[4 * k + 1] * y) + pose[4 * k + 2] * z) + pose[4 * k + 3];
}

/* G3-G4: the segment of the ray s -> p that a ray updates (the truncation band, or with
   whole = 1 the ray from the sensor on), in voxel units A -> B; e = p - s and r = |e|.
   Returns 0 when r = 0 or an end lies outside the voxel range. */
static int ray_segment(const orc_params* P, int whole, const float p[3], const float s32[3], float e[3],
                       float* r_out, float A[3], float B[3]) {
    const float delta = P->trunc, iv = 1.0f / P->voxel_size;
    for (int k = 0; k < 3; ++k) e[k] = p[k] - s32[k];
    float r = sqrtf((e[0] * e[0] + e[1] * e[1]) + e[2] * e[2]);
    *r_out = r;
    if (r == 0.0f) return 0;
    float t0 = whole ? 0.0f : r - delta;
    if (t0 < 0.0f) t0 = 0.0f;
    float t1 = r + delta;
    for (int k = 0; k < 3; ++k) {
        float u = e[k] / r;
        float a = s32[k] + u * t0;
        float b = s32[k] + u * t1;
        A[k] = a * iv;
        B[k] = b * iv;
        if (!(A[k] >= -(float)ORC_VOX_LIMIT && A[k] < (float)ORC_VOX_LIMIT &&
              B[k] >= -(float)ORC_VOX_LIMIT && B[k] < (float)ORC_VOX_LIMIT)) return 0;
    }
    return 1;
}

/* V5: the distance merged into D, clamped to +-delta. */
static double clamp_distance(double d, double d64) { return d < -d64 ? -d64 : (d > d64 ? d64 : d); }

/* Colour of a voxel: the running mean of its rays' colours with the weights of Eq. (3), blended
   with the weight W the voxel held before the frame, stored as an integer per channel (8-bit
   colour), rounded to nearest, ties to even. */
static void fold_color(orc_voxel* vx, double sw, const double swc[3]) {
    for (int k = 0; k < 3; ++k) vx->C[k] = nearbyint((vx->W * vx->C[k] + swc[k]) / (vx->W + sw));
}

/* V6/V8: one frame's update of a voxel by Eqs. (3)-(4), then the storage rounding; swc (NULL:
   colour unchanged) the frame's colour sums of a colour map. */
static void fold_voxel(const orc_params* P, orc_voxel* vx, double sw, double swd, const double* swc) {
    const double wmax = (double)P->w_max;
    if (P->color && swc) fold_color(vx, sw, swc);
    vx->D = (vx->W * vx->D + swd) / (vx->W + sw);
    vx->W = vx->W + sw < wmax ? vx->W + sw : wmax;
    if (P->fp16) {
        vx->D = P->fp16 == 2 ? orc_round_s16(vx->D) : orc_round_half(vx->D);
        vx->W = orc_round_half(vx->W);
    }
}

/* Casts one ray through the truncation band and accumulates its observations. */
static void cast_ray(orc_map* m, const orc_ray* ray, const float s32[3], const double s64[3],
                     orc_stats* st, int32_t* buf, int bufcap) {
    const orc_params* P = &m->P;
    const float v = P->voxel_size, delta = P->trunc;
    /* segment of the ray the update covers, binary32 */
    float e[3], A[3], B[3], r;
    if (!ray_segment(P, P->full_ray, ray->p32, s32, e, &r, A, B)) { st->out_of_bounds++; return; }
    st->rays++;
    int cnt = orc_dda(A, B, buf, bufcap);
    if (cnt > bufcap) cnt = bufcap; /* cannot happen: bufcap covers the longest band */

    const double v64 = (double)v, d64 = (double)delta, eps = v64;
    double es64[3], er = 0.0;
    for (int k = 0; k < 3; ++k) { es64[k] = ray->p64[k] - s64[k]; er += es64[k] * es64[k]; }
    er = sqrt(er);
    for (int i = 0; i < cnt; ++i) {
        const int32_t* g = buf + 3 * i;
        double d;
        if (P->dist == 0) {
            /* Eq. (1): sign decided in binary32, magnitude in binary64 */
            float f0 = ray->p32[0] - ((float)g[0] + 0.5f) * v;
            float f1 = ray->p32[1] - ((float)g[1] + 0.5f) * v;
            float f2 = ray->p32[2] - ((float)g[2] + 0.5f) * v;
            float dot = (f0 * e[0] + f1 * e[1]) + f2 * e[2];
            double sgn = dot > 0.0f ? 1.0 : (dot < 0.0f ? -1.0 : 0.0);
            double n2 = 0.0;
            for (int k = 0; k < 3; ++k) {
                double x = ((double)g[k] + 0.5) * v64;
                double f = ray->p64[k] - x;
                n2 += f * f;
            }
            d = sgn * sqrt(n2);
        } else {
            double dot = 0.0;
            for (int k = 0; k < 3; ++k) {
                double x = ((double)g[k] + 0.5) * v64;
                dot += (ray->p64[k] - x) * es64[k];
            }
            d = dot / er;
        }
        double w = ray->wgt;
        if (P->weighting == 1) w *= dropoff(d, eps, d64);
        double dc = clamp_distance(d, d64);
        int created;
        orc_voxel* vx = (orc_voxel*)table_get(&m->vox, pack3(g[0], g[1], g[2]), 1, &created);
        if (vx->stamp != m->frame + 1) {
            vx->stamp = m->frame + 1;
            vx->sw = 0.0; vx->swd = 0.0; vx->n = 0;
            vx->swc[0] = vx->swc[1] = vx->swc[2] = 0.0;
            add_touch(m, pack3(g[0], g[1], g[2]));
        }
        vx->sw += w;
        vx->swd += w * (dc / d64);
        for (int k = 0; k < 3; ++k) vx->swc[k] += w * ray->col[k];
        vx->n += 1;
        vx->mass += ray->wgt;
        if (P->weighting == 1 && d > -d64 && d <= -eps) vx->ramp += ray->wgt;
        st->touches++;
    }
}

/* Exact mean colour of a group: round(sum Omega c / sum Omega) per channel, to nearest with ties
   to even, in integer arithmetic. */
static double group_color_channel(unsigned __int128 num, uint64_t den) {
    const unsigned __int128 q = num / den, r = num - q * den;
    unsigned __int128 c = q;
    if (2 * r > (unsigned __int128)den || (2 * r == (unsigned __int128)den && (q & 1))) c = q + 1;
    return (double)(uint64_t)c;
}

/*
 * Integrates one frame: points[n][3] in the sensor frame (NaN marks an invalid
 * point), pose[12] = row-major 3x4 T_world_sensor, colors[n] (RGBA8, red in the low byte;
 * NULL: black) for a colour map.  Returns 0.
 */
int orc_integrate_color(orc_map* m, const float* pts, const uint32_t* colors, size_t n, const float pose[12],
                        orc_stats* out);

int orc_integrate(orc_map* m, const float* pts, size_t n, const float pose[12], orc_stats* out) {
    return orc_integrate_color(m, pts, NULL, n, pose, out);
}

int orc_integrate_color(orc_map* m, const float* pts, const uint32_t* colors, size_t n, const float pose[12],
                        orc_stats* out) {
    const orc_params* P = &m->P;
    orc_stats st;
    memset(&st, 0, sizeof st);
    st.points = n;
    const float v = P->voxel_size, iv = 1.0f / v;
    const float rmax2 = P->max_range * P->max_range;
    const float s32[3] = {pose[3], pose[7], pose[11]};
    const double s64[3] = {(double)pose[3], (double)pose[7], (double)pose[11]};
    const int wbits = weight_scale_bits(P);

    /* 1. validity, pose transform and point weight */
    float* p32 = (float*)malloc(n * 3 * sizeof(float) + 1);
    double* p64 = (double*)malloc(n * 3 * sizeof(double) + 1);
    float* w32 = (float*)malloc(n * sizeof(float) + 1);
    double* w64 = (double*)malloc(n * sizeof(double) + 1);
    uint32_t* valid = (uint32_t*)malloc(n * sizeof(uint32_t) + 1);
    size_t nv = 0;
    for (size_t i = 0; i < n; ++i) {
        float x = pts[3 * i], y = pts[3 * i + 1], z = pts[3 * i + 2];
        if (!(isfinite(x) && isfinite(y) && isfinite(z))) { st.invalid++; continue; }
        float rho2 = (x * x + y * y) + z * z;
        if (!(rho2 > 0.0f && rho2 <= rmax2)) { st.invalid++; continue; }
        if (P->weighting == 1 && !(z >= P->z_min)) { st.invalid++; continue; }
        float q[3];
        transform_point(pose, x, y, z, q);
        for (int k = 0; k < 3; ++k)
            p64[3 * nv + k] = (((double)pose[4 * k] * x + (double)pose[4 * k + 1] * y) +
                               (double)pose[4 * k + 2] * z) + (double)pose[4 * k + 3];
        int inside = 1;
        for (int k = 0; k < 3; ++k) {
            float f = q[k] * iv;
            if (!(f >= -(float)ORC_VOX_LIMIT && f < (float)ORC_VOX_LIMIT)) inside = 0;
        }
        if (!inside) { st.out_of_bounds++; continue; }
        for (int k = 0; k < 3; ++k) p32[3 * nv + k] = q[k];
        w32[nv] = P->weighting == 1 ? 1.0f / (z * z) : 1.0f;
        w64[nv] = P->weighting == 1 ? 1.0 / ((double)z * (double)z) : 1.0;
        valid[nv] = (uint32_t)i;
        nv++;
    }
    st.valid = nv;

    /* 2. rays: one per point, or one per group of points sharing a voxel */
    orc_ray* rays = (orc_ray*)malloc((nv + 1) * sizeof(orc_ray));
    size_t nr = 0;
    if (P->merge == 0) {
        for (size_t i = 0; i < nv; ++i) {
            for (int k = 0; k < 3; ++k) {
                rays[nr].p32[k] = p32[3 * i + k];
                rays[nr].p64[k] = P->world64 ? p64[3 * i + k] : (double)p32[3 * i + k];
            }
            rays[nr].wgt = w64[i];
            for (int k = 0; k < 3; ++k)
                rays[nr].col[k] = colors ? (double)((colors[valid[i]] >> (8 * k)) & 255u) : 0.0;
            nr++;
        }
    } else {
        orc_keyidx* ki = (orc_keyidx*)malloc((nv + 1) * sizeof(orc_keyidx));
        for (size_t i = 0; i < nv; ++i) {
            int32_t g[3];
            for (int k = 0; k < 3; ++k) g[k] = (int32_t)floorf(p32[3 * i + k] * iv);
            ki[i].key = pack3(g[0], g[1], g[2]);
            ki[i].idx = (uint32_t)i;
        }
        qsort(ki, nv, sizeof(orc_keyidx), cmp_keyidx);
        float* gp = (float*)malloc((nv + 1) * 3 * sizeof(float));
        float* gw = (float*)malloc((nv + 1) * sizeof(float));
        for (size_t lo = 0; lo < nv;) {
            size_t hi = lo;
            while (hi < nv && ki[hi].key == ki[lo].key) hi++;
            int cnt = (int)(hi - lo);
            double sw = 0.0, sp[3] = {0, 0, 0};
            for (size_t j = lo; j < hi; ++j) {
                uint32_t i = ki[j].idx;
                for (int k = 0; k < 3; ++k) gp[3 * (j - lo) + k] = p32[3 * i + k];
                gw[j - lo] = w32[i];
                sw += w64[i];
                for (int k = 0; k < 3; ++k) sp[k] += w64[i] * p64[3 * i + k];
            }
            orc_group_mean(gp, gw, cnt, v, wbits, rays[nr].p32);
            /* the group's colour: its points' colours weighted as in the mean position */
            unsigned __int128 cs[3] = {0, 0, 0};
            uint64_t cso = 0;
            for (size_t j = lo; j < hi; ++j) {
                const uint32_t i = ki[j].idx;
                const uint64_t om = group_weight(wbits, w32[i]);
                const uint32_t c = colors ? colors[valid[i]] : 0u;
                cso += om;
                for (int k = 0; k < 3; ++k) cs[k] += (unsigned __int128)om * ((c >> (8 * k)) & 255u);
            }
            for (int k = 0; k < 3; ++k) rays[nr].col[k] = group_color_channel(cs[k], cso);
            for (int k = 0; k < 3; ++k) {
                if (P->world64) rays[nr].p64[k] = cnt == 1 ? p64[3 * ki[lo].idx + k] : sp[k] / sw;
                else rays[nr].p64[k] = (double)rays[nr].p32[k];
            }
            rays[nr].wgt = sw;
            nr++;
            lo = hi;
        }
        free(gp); free(gw); free(ki);
    }

    /* 3. raycast the truncation band of every ray */
    m->n_touch = 0;
    const float walk = P->full_ray ? P->max_range + P->trunc : 2.0f * P->trunc;
    int bufcap = 3 * ((int)ceilf(walk / v) + 4) + 8;
    int32_t* buf = (int32_t*)malloc((size_t)bufcap * 3 * sizeof(int32_t));
    for (size_t i = 0; i < nr; ++i) cast_ray(m, &rays[i], s32, s64, &st, buf, bufcap);

    /* 4. Eqs. (3)-(4) once per touched voxel; allocate the blocks of touched voxels */
    for (size_t t = 0; t < m->n_touch; ++t) {
        uint64_t key = m->touch_keys[t];
        orc_voxel* vx = (orc_voxel*)table_get(&m->vox, key, 0, NULL);
        int32_t g[3];
        unpack3(key, &g[0], &g[1], &g[2]);
        int created;
        table_get(&m->blocks, pack3(block_of(g[0]), block_of(g[1]), block_of(g[2])), 1, &created);
        st.new_blocks += (uint64_t)created;
        m->touch_n[t] = vx->n;
        if (vx->sw > 0.0) fold_voxel(P, vx, vx->sw, vx->swd, vx->swc);
    }
    st.voxels = m->n_touch;
    m->frame++;
    m->last = st;
    if (out) *out = st;
    free(buf); free(rays); free(p32); free(p64); free(w32); free(w64); free(valid);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Projection mapping (Sec. IV-B)                                      */
/* ------------------------------------------------------------------ */
/*
 * Integrates one organised frame by projection mapping: instead of casting rays, every voxel
 * of the frame's blocks is projected into the depth image and takes its distance from the
 * depth the image holds at that pixel.
 *  - The blocks: those the truncation bands of the frame's valid points cross (the blocks
 *    raycasting would allocate; every point casts its band, no grouping).
 *  - Geometry (binary32, fixed order, no FMA): the voxel centre x = RN32((g + 1/2) v), its
 *    camera coordinates c_k = ((R_0k e_0 + R_1k e_1) + R_2k e_2) with e = x - t; the pixel
 *    (floor(fx (c_0 / c_2) + cx), floor(fy (c_1 / c_2) + cy)); the voxel is observed when
 *    c_2 > 0, the pixel lies in the image, its point is valid (the validity test of the
 *    point path) and the binary32 distance z_pixel - c_2 exceeds -delta.
 *  - Values (binary64): d = z_pixel - z, z the binary64 depth of the exact voxel centre; the
 *    weight of Eq. (2), or of Eq. (5) with the pixel's depth; D and W by Eqs. (3)-(4) with the
 *    distance clamped to +-delta (one observation per voxel and frame).
 * Reading: the paper names the distance "between the voxel center and the depth value in the
 * image"; it is taken along the optical axis (depth minus depth), as in projective TSDF fusion.
 * Readings of the rest: the image pixel (i, j) holds point i + W j of the organised cloud; the
 * intrinsics map a camera point to pixel coordinates u = fx x / z + cx, v = fy y / z + cy.
 */
int orc_integrate_projective(orc_map* m, const float* pts, size_t n, uint32_t width, const float pose[12],
                             const float intr[4], orc_stats* out) {
    const orc_params* P = &m->P;
    orc_stats st;
    memset(&st, 0, sizeof st);
    st.points = n;
    if (width == 0 || n % width != 0) return -1;
    const uint32_t height = (uint32_t)(n / width);
    const float v = P->voxel_size, iv = 1.0f / v, delta = P->trunc;
    const float rmax2 = P->max_range * P->max_range;
    const float s32[3] = {pose[3], pose[7], pose[11]};

    /* validity of every pixel's point, and the blocks their bands cross */
    uint8_t* ok = (uint8_t*)calloc(n + 1, 1);
    orc_table blocks_now;
    table_init(&blocks_now, 1);
    int bufcap = 3 * ((int)ceilf(2.0f * delta / v) + 4) + 8;
    int32_t* buf = (int32_t*)malloc((size_t)bufcap * 3 * sizeof(int32_t));
    for (size_t i = 0; i < n; ++i) {
        float x = pts[3 * i], y = pts[3 * i + 1], z = pts[3 * i + 2];
        if (!(isfinite(x) && isfinite(y) && isfinite(z))) { st.invalid++; continue; }
        float rho2 = (x * x + y * y) + z * z;
        if (!(rho2 > 0.0f && rho2 <= rmax2)) { st.invalid++; continue; }
        if (P->weighting == 1 && !(z >= P->z_min)) { st.invalid++; continue; }
        float q[3];
        int inside = 1;
        transform_point(pose, x, y, z, q);
        for (int k = 0; k < 3; ++k) {
            float f = q[k] * iv;
            if (!(f >= -(float)ORC_VOX_LIMIT && f < (float)ORC_VOX_LIMIT)) inside = 0;
        }
        if (!inside) { st.out_of_bounds++; continue; }
        ok[i] = 1;
        st.valid++;
        /* the band segment, binary32, as raycasting takes it */
        float e[3], A[3], B[3], r;
        if (!ray_segment(P, 0, q, s32, e, &r, A, B)) { st.out_of_bounds++; continue; }
        st.rays++;
        int cnt = orc_dda(A, B, buf, bufcap);
        if (cnt > bufcap) cnt = bufcap;
        for (int c = 0; c < cnt; ++c) {
            const int32_t* g = buf + 3 * c;
            int created;
            table_get(&blocks_now, pack3(block_of(g[0]), block_of(g[1]), block_of(g[2])), 1, &created);
        }
    }
    free(buf);

    /* every voxel of those blocks, projected */
    const float fx = intr[0], fy = intr[1], cx = intr[2], cy = intr[3];
    double R64[9], t64[3];
    for (int r = 0; r < 3; ++r) {
        for (int c = 0; c < 3; ++c) R64[3 * r + c] = (double)pose[4 * r + c];
        t64[r] = (double)pose[4 * r + 3];
    }
    const double v64 = (double)v, d64 = (double)delta, eps = v64;
    m->n_touch = 0;
    for (size_t bi = 0; bi < blocks_now.cap; ++bi) {
        if (!blocks_now.keys[bi]) continue;
        int32_t bc[3];
        unpack3(blocks_now.keys[bi] - 1, &bc[0], &bc[1], &bc[2]);
        int created;
        table_get(&m->blocks, blocks_now.keys[bi] - 1, 1, &created);
        st.new_blocks += (uint64_t)created;
        for (int l = 0; l < 4096; ++l) {
            const int32_t g[3] = {16 * bc[0] + (l & 15), 16 * bc[1] + ((l >> 4) & 15), 16 * bc[2] + (l >> 8)};
            float e[3], cam[3];
            for (int k = 0; k < 3; ++k) e[k] = ((float)g[k] + 0.5f) * v - s32[k];
            for (int k = 0; k < 3; ++k) cam[k] = (pose[k] * e[0] + pose[4 + k] * e[1]) + pose[8 + k] * e[2];
            if (!(cam[2] > 0.0f)) continue;
            const float uf = fx * (cam[0] / cam[2]) + cx;
            const float vf = fy * (cam[1] / cam[2]) + cy;
            if (!(uf >= 0.0f && uf < (float)width && vf >= 0.0f && vf < (float)height)) continue;
            const size_t pix = (size_t)floorf(uf) + (size_t)width * (size_t)floorf(vf);
            if (!ok[pix]) continue;
            const float zm = pts[3 * pix + 2];
            if (!(zm - cam[2] > -delta)) continue;
            /* values, binary64: depth of the exact centre */
            double z = 0.0;
            for (int k = 0; k < 3; ++k) z += R64[3 * k + 2] * (((double)g[k] + 0.5) * v64 - t64[k]);
            const double d = (double)zm - z;
            double w = P->weighting == 1 ? 1.0 / ((double)zm * (double)zm) : 1.0;
            const double wgt = w;
            if (P->weighting == 1) w *= dropoff(d, eps, d64);
            const double dc = clamp_distance(d, d64);
            orc_voxel* vx = (orc_voxel*)table_get(&m->vox, pack3(g[0], g[1], g[2]), 1, &created);
            add_touch(m, pack3(g[0], g[1], g[2]));
            m->touch_n[m->n_touch - 1] = 1;
            vx->mass += wgt;
            if (P->weighting == 1 && d > -d64 && d <= -eps) vx->ramp += wgt;
            st.touches++;
            if (w > 0.0) fold_voxel(P, vx, w, w * (dc / d64), NULL);   /* colour: raycasting only */
        }
    }
    st.voxels = m->n_touch;
    m->frame++;
    m->last = st;
    if (out) *out = st;
    table_free(&blocks_now);
    free(ok);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Export                                                              */
/* ------------------------------------------------------------------ */
size_t orc_num_blocks(const orc_map* m) { return m->blocks.size; }

static int cmp_u64(const void* a, const void* b) {
    uint64_t x = *(const uint64_t*)a, y = *(const uint64_t*)b;
    return x < y ? -1 : (x > y);
}

/*
 * Writes the blocks in ascending (bx, by, bz) order: coords[cap][3], and per block
 * 4096 voxels (x fastest) of D (metres), W and the sum of ray weights seen.
 * Any of the arrays may be NULL.  Returns the number of blocks.
 */
size_t orc_export(const orc_map* m, int32_t* coords, double* D, double* W, double* mass, size_t cap) {
    size_t nb = m->blocks.size;
    uint64_t* keys = (uint64_t*)malloc((nb + 1) * sizeof(uint64_t));
    size_t j = 0;
    for (size_t i = 0; i < m->blocks.cap; ++i)
        if (m->blocks.keys[i]) keys[j++] = m->blocks.keys[i] - 1;
    qsort(keys, nb, sizeof(uint64_t), cmp_u64);
    const double d64 = (double)m->P.trunc;
    for (size_t b = 0; b < nb && b < cap; ++b) {
        int32_t bc[3];
        unpack3(keys[b], &bc[0], &bc[1], &bc[2]);
        if (coords) { coords[3 * b] = bc[0]; coords[3 * b + 1] = bc[1]; coords[3 * b + 2] = bc[2]; }
        for (int l = 0; l < 4096; ++l) {
            int32_t g0 = 16 * bc[0] + (l & 15), g1 = 16 * bc[1] + ((l >> 4) & 15), g2 = 16 * bc[2] + (l >> 8);
            const orc_voxel* vx = (const orc_voxel*)table_get((orc_table*)&m->vox, pack3(g0, g1, g2), 0, NULL);
            size_t o = b * 4096 + (size_t)l;
            if (D) D[o] = vx ? vx->D * d64 : 0.0;
            if (W) W[o] = vx ? vx->W : 0.0;
            if (mass) mass[o] = vx ? vx->mass : 0.0;
        }
    }
    free(keys);
    return nb;
}

/*
 * Per voxel, in orc_export's order: the summed weight of the rays that saw the voxel on the
 * Eq. (5) ramp.  D's sensitivity to distance rounding grows with it (the ramp weights move
 * with the distance).  Returns the number of blocks.
 */
size_t orc_export_ramp(const orc_map* m, double* ramp, size_t cap) {
    size_t nb = m->blocks.size;
    uint64_t* keys = (uint64_t*)malloc((nb + 1) * sizeof(uint64_t));
    size_t j = 0;
    for (size_t i = 0; i < m->blocks.cap; ++i)
        if (m->blocks.keys[i]) keys[j++] = m->blocks.keys[i] - 1;
    qsort(keys, nb, sizeof(uint64_t), cmp_u64);
    for (size_t b = 0; b < nb && b < cap; ++b) {
        int32_t bc[3];
        unpack3(keys[b], &bc[0], &bc[1], &bc[2]);
        for (int l = 0; l < 4096; ++l) {
            int32_t g0 = 16 * bc[0] + (l & 15), g1 = 16 * bc[1] + ((l >> 4) & 15), g2 = 16 * bc[2] + (l >> 8);
            const orc_voxel* vx = (const orc_voxel*)table_get((orc_table*)&m->vox, pack3(g0, g1, g2), 0, NULL);
            ramp[b * 4096 + (size_t)l] = vx ? vx->ramp : 0.0;
        }
    }
    free(keys);
    return nb;
}

/* Colours of every voxel in orc_export's order, packed RGB8 (red in the low byte; 0 where the
   voxel was never observed).  Returns the number of blocks. */
size_t orc_export_color(const orc_map* m, uint32_t* rgb, size_t cap) {
    size_t nb = m->blocks.size;
    uint64_t* keys = (uint64_t*)malloc((nb + 1) * sizeof(uint64_t));
    size_t j = 0;
    for (size_t i = 0; i < m->blocks.cap; ++i)
        if (m->blocks.keys[i]) keys[j++] = m->blocks.keys[i] - 1;
    qsort(keys, nb, sizeof(uint64_t), cmp_u64);
    for (size_t b = 0; b < nb && b < cap; ++b) {
        int32_t bc[3];
        unpack3(keys[b], &bc[0], &bc[1], &bc[2]);
        for (int l = 0; l < 4096; ++l) {
            int32_t g0 = 16 * bc[0] + (l & 15), g1 = 16 * bc[1] + ((l >> 4) & 15), g2 = 16 * bc[2] + (l >> 8);
            const orc_voxel* vx = (const orc_voxel*)table_get((orc_table*)&m->vox, pack3(g0, g1, g2), 0, NULL);
            uint32_t c = 0;
            if (vx)
                for (int k = 0; k < 3; ++k) c |= (uint32_t)vx->C[k] << (8 * k);
            rgb[b * 4096 + (size_t)l] = c;
        }
    }
    free(keys);
    return nb;
}

/* Touches of the last frame: voxel coordinates [cap][3] and ray counts. Returns the count. */
size_t orc_last_touches(const orc_map* m, int32_t* coords, uint32_t* counts, size_t cap) {
    for (size_t t = 0; t < m->n_touch && t < cap; ++t) {
        unpack3(m->touch_keys[t], &coords[3 * t], &coords[3 * t + 1], &coords[3 * t + 2]);
        counts[t] = m->touch_n[t];
    }
    return m->n_touch;
}

void orc_last_stats(const orc_map* m, orc_stats* out) { *out = m->last; }
