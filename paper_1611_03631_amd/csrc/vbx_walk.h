// Voxel traversal of a segment (Amanatides-Woo stepping in binary32, a fixed operation order)
// and the sequence of 16^3 blocks it passes through.  Pure arithmetic: the kernels use it, and
// the host check of the block sequence (tests/walk_check.cpp) compiles it with a host compiler.
#pragma once

#ifdef __HIPCC__
#define VBX_HD __host__ __device__
#else
#define VBX_HD
#endif

#ifdef __clang__
#pragma clang fp contract(off)
#endif

namespace vbx {

struct Walk {
    int g[3];        // current voxel
    int n[3];        // steps left per axis
    int step[3];
    float tM[3], tD[3];
    int left;        // total steps left
};

// Traversal from voxel-space end points A -> B: the voxel of A, then one voxel per crossed
// face.  tM[k] is the segment parameter of axis k's next face crossing, tD[k] its increment.
VBX_HD inline void walk_setup_vox(const float A[3], const float B[3], Walk& w) {
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
}

// One step: among axes with steps left, the smallest crossing parameter; ties go
// to the lowest axis.
// (Constant indices only, so the walk state stays in registers.)
VBX_HD inline void walk_step(Walk& w) {
    // the axis with steps left whose next boundary comes first (ties: the lowest axis), chosen
    // with selects rather than branches (bitwise operators: no short-circuit), so that the lanes
    // of a wave never diverge here
    const bool c0 = w.n[0] > 0, c1 = w.n[1] > 0, c2 = w.n[2] > 0;
    const bool t1 = c1 & (!c0 | (w.tM[1] < w.tM[0]));
    const float best = t1 ? w.tM[1] : w.tM[0];
    const bool t2 = c2 & ((!c0 & !t1) | (w.tM[2] < best));
    // an axis is always found: the caller only steps while w.left > 0
    const int axis = t2 ? 2 : (t1 ? 1 : 0);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const bool s = axis == k;
        const float next = w.tM[k] + w.tD[k];
        w.g[k] += s ? w.step[k] : 0;
        w.n[k] -= s ? 1 : 0;
        w.tM[k] = s ? next : w.tM[k];
    }
    w.left -= 1;
}

// ---------------------------------------------------------------------------
// Blocks of a traversal without its voxels
// ---------------------------------------------------------------------------
// The steps of axis k carry the parameters t_k(0) = tM[k], t_k(j + 1) = t_k(j) + tD[k] (each sum
// rounded), strictly increasing.  Each step of the walk takes the smallest parameter among the
// axes' next steps, ties to the lowest axis, so the walk takes all its steps in increasing order
// of (parameter, axis).  The block changes on the steps that carry g_k across a multiple of 16,
// every 16th step of an axis; their order, and so the block sequence, follows from their own
// parameters, formed by the same additions as the voxel walk's.
struct BlockWalk {
    int b[3];      // current block (voxel index >> 4)
    int step[3];
    int ev[3];     // index among axis k's steps of its next block-changing step
    int n[3];      // axis k's steps in the whole walk
    float T[3];    // parameter of that step; +inf when the axis changes block no more
    float tD[3];
};

// The block of the walk's first voxel and each axis' first block-changing step.
VBX_HD inline void block_walk_init(const Walk& w, BlockWalk& bw) {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        bw.b[k] = w.g[k] >> 4;   // arithmetic shift: floor division by 16
        bw.step[k] = w.step[k];
        bw.n[k] = w.n[k];
        bw.tD[k] = w.tD[k];
        // steps before the one that leaves the block: up to the block's last voxel going up,
        // down to its first going down
        const int e = w.step[k] > 0 ? 15 - (w.g[k] & 15) : (w.g[k] & 15);
        bw.ev[k] = e;
        float t = __builtin_inff();
        if (e < w.n[k]) {
            t = w.tM[k];
            for (int j = 0; j < e; ++j) t = t + w.tD[k];
        }
        bw.T[k] = t;
    }
}

// Takes the walk's next block-changing step: returns its axis, with b[] the new block, or -1
// when the walk changes block no more.
VBX_HD inline int block_walk_next(BlockWalk& bw) {
    const bool t1 = bw.T[1] < bw.T[0];
    const float best = t1 ? bw.T[1] : bw.T[0];
    const bool t2 = bw.T[2] < best;
    const int axis = t2 ? 2 : (t1 ? 1 : 0);
    const float cur = t2 ? bw.T[2] : best;
    if (!(cur < __builtin_inff())) return -1;
    // the chosen axis' parameter and increment, then its block-changing step 16 steps on
    const float inc = axis == 0 ? bw.tD[0] : (axis == 1 ? bw.tD[1] : bw.tD[2]);
    const int evn = (axis == 0 ? bw.ev[0] : (axis == 1 ? bw.ev[1] : bw.ev[2])) + 16;
    const int na = axis == 0 ? bw.n[0] : (axis == 1 ? bw.n[1] : bw.n[2]);
    float t = __builtin_inff();
    if (evn < na) {
        t = cur;
        for (int j = 0; j < 16; ++j) t = t + inc;
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const bool s = axis == k;
        bw.b[k] += s ? bw.step[k] : 0;
        bw.ev[k] = s ? evn : bw.ev[k];
        bw.T[k] = s ? t : bw.T[k];
    }
    return axis;
}

}  // namespace vbx
