// Host check of the block sequence of a traversal (vbx_walk.h): the blocks found from the
// block-changing steps alone (block_walk_init / block_walk_next) must be the distinct blocks of
// the voxel walk (walk_setup_vox / walk_step), in order, for every segment.  Built with the host
// compiler by tests/test_walk_host.py; prints "ALL OK" or the first differing segment.
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "vbx_walk.h"

using vbx::BlockWalk;
using vbx::Walk;

struct Blk {
    int b[3];
    bool operator==(const Blk& o) const { return b[0] == o.b[0] && b[1] == o.b[1] && b[2] == o.b[2]; }
};

static std::vector<Blk> by_voxels(const float A[3], const float B[3], long* steps) {
    Walk w;
    vbx::walk_setup_vox(A, B, w);
    std::vector<Blk> out;
    for (;;) {
        const Blk c = {{w.g[0] >> 4, w.g[1] >> 4, w.g[2] >> 4}};
        if (out.empty() || !(out.back() == c)) out.push_back(c);
        if (w.left == 0) break;
        vbx::walk_step(w);
        ++*steps;
    }
    return out;
}

static std::vector<Blk> by_blocks(const float A[3], const float B[3]) {
    Walk w;
    vbx::walk_setup_vox(A, B, w);
    BlockWalk bw;
    vbx::block_walk_init(w, bw);
    std::vector<Blk> out;
    for (int axis = 0; axis >= 0; axis = vbx::block_walk_next(bw)) out.push_back({{bw.b[0], bw.b[1], bw.b[2]}});
    return out;
}

static long n_checked = 0, n_multi = 0, n_steps = 0;

static void check(const float A[3], const float B[3]) {
    const std::vector<Blk> a = by_voxels(A, B, &n_steps), b = by_blocks(A, B);
    ++n_checked;
    if (a.size() > 1) ++n_multi;
    if (!(a == b)) {
        std::printf("MISMATCH A=(%.9g %.9g %.9g) B=(%.9g %.9g %.9g): %zu blocks by voxels, %zu by block steps\n",
                    A[0], A[1], A[2], B[0], B[1], B[2], a.size(), b.size());
        for (const Blk& x : a) std::printf("  v (%d %d %d)\n", x.b[0], x.b[1], x.b[2]);
        for (const Blk& x : b) std::printf("  b (%d %d %d)\n", x.b[0], x.b[1], x.b[2]);
        std::exit(1);
    }
}

int main() {
    std::mt19937_64 rng(1234567);
    std::uniform_real_distribution<float> U(-1.0f, 1.0f);
    float A[3], B[3];
    // band-length and longer segments anywhere
    for (int i = 0; i < 1500000; ++i) {
        const float len = i % 3 == 0 ? 30.0f : (i % 3 == 1 ? 80.0f : 400.0f);
        for (int k = 0; k < 3; ++k) {
            A[k] = 300.0f * U(rng);
            B[k] = A[k] + len * U(rng);
        }
        check(A, B);
    }
    // dyadic end points on and near block faces, edges and corners: exact ties of the crossing
    // parameters between axes
    std::uniform_int_distribution<int> Ib(-6, 6), If(-8, 8), Il(-48, 48);
    for (int i = 0; i < 1500000; ++i) {
        for (int k = 0; k < 3; ++k) {
            A[k] = 16.0f * (float)Ib(rng) + (float)If(rng) * 0.25f;
            B[k] = A[k] + (float)Il(rng) * 0.5f;
        }
        check(A, B);
    }
    // segments through block corners, symmetric about them, and axis-aligned ones
    for (int i = 0; i < 500000; ++i) {
        const float c[3] = {16.0f * (float)Ib(rng), 16.0f * (float)Ib(rng), 16.0f * (float)Ib(rng)};
        float d[3];
        for (int k = 0; k < 3; ++k) d[k] = (float)Il(rng) * 0.125f;
        const int axis_only = i % 7 == 0 ? (i / 7) % 3 : -1;
        for (int k = 0; k < 3; ++k) {
            const float dk = axis_only >= 0 && k != axis_only ? 0.0f : d[k];
            A[k] = c[k] - dk + (axis_only >= 0 && k != axis_only ? 0.5f : 0.0f);
            B[k] = c[k] + dk + (axis_only >= 0 && k != axis_only ? 0.5f : 0.0f);
        }
        check(A, B);
    }
    // zero-length and one-voxel segments
    for (int i = 0; i < 100000; ++i) {
        for (int k = 0; k < 3; ++k) {
            A[k] = 100.0f * U(rng);
            B[k] = i % 2 ? A[k] : A[k] + 0.01f * U(rng);
        }
        check(A, B);
    }
    std::printf("%ld segments (%ld crossing blocks, %ld voxel steps): ALL OK\n", n_checked, n_multi, n_steps);
    return 0;
}
