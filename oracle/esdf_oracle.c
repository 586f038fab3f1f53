/*
 * CPU oracle for building a Euclidean signed distance field (ESDF) from a TSDF
 * (Oleynikova et al., "Voxblox", Sec. V-A "Construction", Algorithm 1).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library may include, link,
 * load or call this file: only the test-suite and the CPU baseline leg of the
 * benchmark use it.  It shares no code with the GPU path.
 *
 * Plain and serial: a hash map from voxel index to ESDF voxel, two queues, and
 * the steps of Algorithm 1 in the order the paper gives them, in binary64.
 *
 * What a call computes.  Given the TSDF voxels that changed (index, distance d_T,
 * weight W_T; W_T = 0 is an unknown voxel and is skipped), every changed voxel is
 * first classified: it is *fixed* when |d_T| < gamma (the fixed band around the
 * surface takes its value from the TSDF and is never modified by the waves).
 *  - fixed: an unobserved voxel takes d_T and enters the lower queue; an observed one
 *    takes d_T and enters both the raise and the lower queue;
 *  - not fixed: a voxel that was fixed, or whose TSDF distance changed sign, becomes
 *    sign(d_T) d_max and enters the raise queue; an unobserved voxel becomes sign(d_T) d_max and puts its observed
 *    neighbours in the lower queue; an observed voxel that was not fixed is left.
 * Then the raise queue is emptied (a popped voxel that is not fixed returns to
 * sign(d) d_max and loses its parent; each observed neighbour is raised when its
 * parent is the popped voxel, else lowered), then the lower queue (a popped voxel
 * offers every observed, non-fixed neighbour its distance plus the step length;
 * the neighbour takes it when it is smaller in magnitude, with the popped voxel as
 * its parent, and is queued).
 *
 * Readings (the paper's listing leaves these open or is at odds with its text):
 *  - 26-connectivity with quasi-Euclidean step lengths v, sqrt(2) v, sqrt(3) v.
 *  - Fixed voxels are never changed by either wave (the text says they may not
 *    be modified; the listing's raise step would reset them).
 *  - Unknown voxels (never observed in the TSDF) are neither updated nor used to
 *    propagate (the text); the listing's "each neighbour" means each observed one.
 *  - A voxel outside the band keeps the sign its TSDF distance had when it was
 *    first observed or left the band (its side of the surface): the lower wave offers a positive voxel max(d + dist, 0)
 *    and a negative one min(d - dist, 0) (the listing's two conditions, with a
 *    candidate that would cross zero stopped at zero).  Distances cross the surface
 *    only from fixed voxels, the band that stands for it: a voxel that is not fixed
 *    passes its distance to voxels on its own side only.  (Across a gap in the band
 *    the listing would hand a positive voxel the distance of a negative one that is
 *    still moving towards zero, and the field would depend on the queue order.)
 *  - The parent is stored as the direction from a voxel to its parent; a
 *    neighbour is the popped voxel's child when its parent direction points back at
 *    the popped voxel.
 *  - The fixed flag of the ESDF voxel follows |d_T| < gamma at every update.
 *  - The listing leaves an observed voxel outside the band alone.  One whose TSDF
 *    distance changed sign (without passing through the band) is treated as a voxel
 *    that left the band, so that its side follows the TSDF and the voxels that took
 *    their distance from it on the old side are raised.
 *  - The listing sends a fixed voxel whose distance decreased to the lower queue
 *    only.  That holds for unsigned distances; with signed ones a voxel whose value
 *    decreases moves its negative dependents away from zero, which only a raise
 *    undoes.  So every observed voxel that enters (or stays in) the fixed band
 *    is raised and lowered, and only a newly observed one is lowered alone.
 * The queue is a FIFO or a bucketed priority queue on |d| (single insertion while
 * queued); both reach the same distances, which the pins check.
 *
 * Build: gcc -O2 -std=gnu11 -ffp-contract=off (binary64 arithmetic throughout).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ */
/* Voxels                                                              */
/* ------------------------------------------------------------------ */
typedef struct {
    double d;          /* signed distance (metres) */
    uint8_t observed;
    uint8_t fixed;
    int8_t parent;     /* neighbour index 0..26 (13 = none) of the parent, as seen from this voxel */
    uint8_t queued;    /* in the lower queue (priority mode: single insertion) */
    uint8_t neg;       /* side of the surface: 1 when first observed with d_T < 0 */
} esdf_vox;

typedef struct {
    uint64_t* keys;    /* key + 1, 0 = empty */
    esdf_vox* vals;
    size_t cap, size;
} vox_table;

static uint64_t hash64(uint64_t x) {
    x ^= x >> 31; x *= 0x7fb5d329728ea185ULL;
    x ^= x >> 27; x *= 0x81dadef4bc2dd44dULL;
    x ^= x >> 33;
    return x;
}

static uint64_t vkey(int32_t x, int32_t y, int32_t z) {
    return ((uint64_t)(uint32_t)(x + (1 << 20)) << 42) | ((uint64_t)(uint32_t)(y + (1 << 20)) << 21) |
           (uint64_t)(uint32_t)(z + (1 << 20));
}
static void vunkey(uint64_t k, int32_t g[3]) {
    g[0] = (int32_t)((k >> 42) & 0x1FFFFF) - (1 << 20);
    g[1] = (int32_t)((k >> 21) & 0x1FFFFF) - (1 << 20);
    g[2] = (int32_t)(k & 0x1FFFFF) - (1 << 20);
}

static esdf_vox* vt_get(vox_table* t, uint64_t key, int create);

static void vt_grow(vox_table* t) {
    vox_table n;
    n.cap = t->cap ? 2 * t->cap : 4096;
    n.size = 0;
    n.keys = (uint64_t*)calloc(n.cap, sizeof(uint64_t));
    n.vals = (esdf_vox*)calloc(n.cap, sizeof(esdf_vox));
    for (size_t i = 0; i < t->cap; ++i)
        if (t->keys[i]) *vt_get(&n, t->keys[i] - 1, 1) = t->vals[i];
    free(t->keys);
    free(t->vals);
    *t = n;
}

static esdf_vox* vt_get(vox_table* t, uint64_t key, int create) {
    if (create && 2 * (t->size + 1) > t->cap) vt_grow(t);
    if (!t->cap) return NULL;
    size_t mask = t->cap - 1, i = (size_t)hash64(key) & mask;
    for (;;) {
        if (t->keys[i] == key + 1) return &t->vals[i];
        if (!t->keys[i]) {
            if (!create) return NULL;
            t->keys[i] = key + 1;
            memset(&t->vals[i], 0, sizeof(esdf_vox));
            t->vals[i].parent = 13;
            t->size++;
            return &t->vals[i];
        }
        i = (i + 1) & mask;
    }
}

/* ------------------------------------------------------------------ */
/* Queues                                                              */
/* ------------------------------------------------------------------ */
typedef struct {
    uint64_t* a;
    size_t head, tail, cap;   /* ring buffer */
} fifo;

static void fifo_push(fifo* q, uint64_t k) {
    if (q->tail - q->head == q->cap) {
        size_t nc = q->cap ? 2 * q->cap : 1024;
        uint64_t* na = (uint64_t*)malloc(nc * sizeof(uint64_t));
        for (size_t i = q->head; i < q->tail; ++i) na[i - q->head] = q->a[i % q->cap];
        free(q->a);
        q->a = na;
        q->tail -= q->head;
        q->head = 0;
        q->cap = nc;
    }
    q->a[q->tail % q->cap] = k;
    q->tail++;
}
static int fifo_pop(fifo* q, uint64_t* k) {
    if (q->head == q->tail) return 0;
    *k = q->a[q->head % q->cap];
    q->head++;
    return 1;
}

/* Bucketed priority queue on |d|: bucket floor(|d| / width), lowest bucket first, FIFO
   within a bucket. */
typedef struct {
    fifo* b;
    size_t nb, lowest, count;
    double width;
} bucketq;

static void bq_push(bucketq* q, uint64_t k, double absd) {
    size_t i = (size_t)(absd / q->width);
    if (i >= q->nb) i = q->nb - 1;
    fifo_push(&q->b[i], k);
    if (i < q->lowest) q->lowest = i;
    q->count++;
}
static int bq_pop(bucketq* q, uint64_t* k) {
    if (!q->count) return 0;
    while (q->b[q->lowest].head == q->b[q->lowest].tail) q->lowest++;
    fifo_pop(&q->b[q->lowest], k);
    q->count--;
    return 1;
}

/* ------------------------------------------------------------------ */
/* The ESDF                                                            */
/* ------------------------------------------------------------------ */
typedef struct {
    double v, gamma, d_max;
    int priority;          /* 0: FIFO lower queue; 1: bucketed priority queue */
    vox_table vox;
    fifo raise;
    fifo lower_fifo;
    bucketq lower_pq;
    uint64_t pops_raise, pops_lower, updates;
} orc_esdf;

/* neighbour index n in 0..26 (13 = the voxel itself) <-> offset */
static void offset_of(int n, int o[3]) { o[0] = n % 3 - 1; o[1] = (n / 3) % 3 - 1; o[2] = n / 9 - 1; }

static double step_length(const orc_esdf* E, int n) {
    int o[3];
    offset_of(n, o);
    const int k = o[0] * o[0] + o[1] * o[1] + o[2] * o[2];
    return E->v * sqrt((double)k);      /* v, sqrt(2) v, sqrt(3) v */
}

orc_esdf* orc_esdf_create(double voxel_size, double gamma, double d_max, int priority) {
    orc_esdf* E = (orc_esdf*)calloc(1, sizeof(orc_esdf));
    E->v = voxel_size;
    E->gamma = gamma;
    E->d_max = d_max;
    E->priority = priority;
    E->lower_pq.width = voxel_size / 4.0;
    E->lower_pq.nb = (size_t)(d_max / E->lower_pq.width) + 2;
    E->lower_pq.b = (fifo*)calloc(E->lower_pq.nb, sizeof(fifo));
    E->lower_pq.lowest = E->lower_pq.nb;
    return E;
}

void orc_esdf_destroy(orc_esdf* E) {
    if (!E) return;
    free(E->vox.keys);
    free(E->vox.vals);
    free(E->raise.a);
    free(E->lower_fifo.a);
    for (size_t i = 0; i < E->lower_pq.nb; ++i) free(E->lower_pq.b[i].a);
    free(E->lower_pq.b);
    free(E);
}

static double sgn(double x) { return x > 0.0 ? 1.0 : (x < 0.0 ? -1.0 : 0.0); }

static void insert_lower(orc_esdf* E, uint64_t k) {
    esdf_vox* x = vt_get(&E->vox, k, 0);
    if (!x || !x->observed) return;
    if (E->priority) {
        if (x->queued) return;
        x->queued = 1;
        bq_push(&E->lower_pq, k, fabs(x->d));
    } else {
        fifo_push(&E->lower_fifo, k);
    }
}

static int pop_lower(orc_esdf* E, uint64_t* k) {
    if (E->priority) {
        if (!bq_pop(&E->lower_pq, k)) return 0;
        vt_get(&E->vox, *k, 0)->queued = 0;
        return 1;
    }
    return fifo_pop(&E->lower_fifo, k);
}

static uint64_t neighbour_key(uint64_t k, int n) {
    int32_t g[3];
    int o[3];
    vunkey(k, g);
    offset_of(n, o);
    return vkey(g[0] + o[0], g[1] + o[1], g[2] + o[2]);
}

static void process_raise(orc_esdf* E) {
    uint64_t k;
    while (fifo_pop(&E->raise, &k)) {
        E->pops_raise++;
        esdf_vox* x = vt_get(&E->vox, k, 0);
        if (!x->fixed) {
            x->d = (x->neg ? -1.0 : 1.0) * E->d_max;
            x->parent = 13;
        }
        for (int n = 0; n < 27; ++n) {
            if (n == 13) continue;
            const uint64_t nk = neighbour_key(k, n);
            esdf_vox* y = vt_get(&E->vox, nk, 0);
            if (!y || !y->observed) continue;
            /* y is a child of x when y's parent direction points back at x */
            if (!y->fixed && y->parent == 26 - n) fifo_push(&E->raise, nk);
            else insert_lower(E, nk);
        }
    }
}

static void process_lower(orc_esdf* E) {
    uint64_t k;
    while (pop_lower(E, &k)) {
        E->pops_lower++;
        const esdf_vox* x = vt_get(&E->vox, k, 0);
        const double dx = x->d;
        for (int n = 0; n < 27; ++n) {
            if (n == 13) continue;
            const uint64_t nk = neighbour_key(k, n);
            esdf_vox* y = vt_get(&E->vox, nk, 0);
            if (!y || !y->observed || y->fixed) continue;
            if (!x->fixed && x->neg != y->neg) continue;     /* only the band crosses the surface */
            const double dist = step_length(E, n);
            double c;
            int better;
            if (!y->neg) {
                c = dx + dist;
                if (c < 0.0) c = 0.0;
                better = c < y->d;
            } else {
                c = dx - dist;
                if (c > 0.0) c = 0.0;
                better = c > y->d;
            }
            if (better) {
                y->d = c;
                y->parent = (int8_t)(26 - n);      /* from y towards x */
                E->updates++;
                insert_lower(E, nk);
            }
        }
    }
}

/*
 * One update (Algorithm 1, Propagate): coords[n][3] voxel indices of the TSDF voxels that
 * changed, d[n] their TSDF distance (metres) and w[n] their weight (0: unknown, skipped).
 */
void orc_esdf_update(orc_esdf* E, size_t n, const int32_t* coords, const double* d, const double* w) {
    for (size_t i = 0; i < n; ++i) {
        if (!(w[i] > 0.0)) continue;
        const uint64_t k = vkey(coords[3 * i], coords[3 * i + 1], coords[3 * i + 2]);
        esdf_vox* x = vt_get(&E->vox, k, 1);
        const double dt = d[i];
        if (-E->gamma < dt && dt < E->gamma) {            /* isFixed */
            if (!x->observed) {
                x->observed = 1;
                x->neg = dt < 0.0;
                x->fixed = 1;
                x->d = dt;
                x->parent = 13;
                insert_lower(E, k);
            } else {
                x->fixed = 1;
                x->neg = dt < 0.0;       /* a band voxel's side is the sign of its value */
                x->d = dt;
                x->parent = 13;
                fifo_push(&E->raise, k);
                insert_lower(E, k);
            }
        } else if (x->fixed || (x->observed && (dt < 0.0) != (x->neg != 0))) {
            /* left the band, or changed side outside it */
            x->fixed = 0;
            x->observed = 1;
            x->neg = dt < 0.0;
            x->d = sgn(dt) * E->d_max;
            x->parent = 13;
            fifo_push(&E->raise, k);
        } else if (!x->observed) {
            x->observed = 1;
            x->neg = dt < 0.0;
            x->d = sgn(dt) * E->d_max;
            x->parent = 13;
            for (int m = 0; m < 27; ++m)
                if (m != 13) insert_lower(E, neighbour_key(k, m));
        }
    }
    process_raise(E);
    process_lower(E);
}

/* Observed voxels: coords [cap][3], d [cap], info [cap] (bit 0 observed, bit 1 fixed, bits
   2..6 parent index 0..26 with 13 = none, bit 7 negative side).  Returns the number of
   observed voxels. */
size_t orc_esdf_export(const orc_esdf* E, int32_t* coords, double* d, uint8_t* info, size_t cap) {
    size_t j = 0;
    for (size_t i = 0; i < E->vox.cap; ++i) {
        if (!E->vox.keys[i] || !E->vox.vals[i].observed) continue;
        if (j < cap) {
            if (coords) vunkey(E->vox.keys[i] - 1, coords + 3 * j);
            if (d) d[j] = E->vox.vals[i].d;
            if (info)
                info[j] = (uint8_t)(1u | (E->vox.vals[i].fixed ? 2u : 0u) | ((uint8_t)E->vox.vals[i].parent << 2) |
                                    (E->vox.vals[i].neg ? 128u : 0u));
        }
        j++;
    }
    return j;
}

void orc_esdf_counts(const orc_esdf* E, uint64_t out[3]) {
    out[0] = E->pops_raise;
    out[1] = E->pops_lower;
    out[2] = E->updates;
}
