// Host checks of the map server's scheduling core (admission, tick formation, per-map order,
// replay after a full pool), run against a fake executor.  Built with the host compiler by
// tests/test_sched_host.py; exits non-zero on the first failed check.
#include <cstdio>
#include <cstdlib>
#include <map>
#include <random>
#include <vector>

#include "vbx_sched.h"

using vbx_sched::Planner;
using vbx_sched::Request;

#define CHECK(c)                                                             \
    do {                                                                     \
        if (!(c)) {                                                          \
            std::fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c); \
            std::exit(1);                                                    \
        }                                                                    \
    } while (0)

static std::vector<uint64_t> tickets(const std::vector<Request*>& v) {
    std::vector<uint64_t> t;
    for (const Request* r : v) t.push_back(r->ticket);
    return t;
}

static void admission() {
    Planner p(1000);
    int a = -1, b = -1, c = -1;
    CHECK(p.admit(400, &a) && a == 0);
    CHECK(p.admit(500, &b) && b == 1);
    CHECK(!p.admit(200, &c) && c == -1);
    CHECK(p.used() == 900 && p.num_maps() == 2);
    CHECK(p.grow(a, 100) && p.used() == 1000);
    CHECK(!p.grow(b, 1) && p.used() == 1000);
    p.release(a, 100);
    CHECK(p.used() == 900 && p.map(a).bytes == 400);
    std::puts("admission ok");
}

static void tick_formation() {
    Planner p(1 << 20);
    int id;
    for (int i = 0; i < 3; ++i) p.admit(1, &id);
    std::vector<Request> R(8);
    const int maps[8] = {0, 1, 0, 2, 1, 0, 2, 2};
    const uint64_t pts[8] = {10, 20, 30, 40, 500, 5, 5, 5};
    for (int i = 0; i < 8; ++i) {
        R[i].ticket = (uint64_t)i + 1;
        R[i].map = maps[i];
        R[i].points = pts[i];
        p.submit(&R[i]);
    }
    // frame limit, in ticket order
    auto t1 = p.next_tick(3, 1000, 8);
    CHECK((tickets(t1) == std::vector<uint64_t>{1, 2, 3}));
    CHECK(p.map(0).inflight == 1 && p.map(1).inflight == 1 && p.map(2).inflight == 0);
    // point limit closes the tick before ticket 5 (500 points); later requests wait too
    auto t2 = p.next_tick(8, 100, 8);
    CHECK((tickets(t2) == std::vector<uint64_t>{4}));
    // a request over the point limit runs alone
    auto t3 = p.next_tick(8, 100, 8);
    CHECK((tickets(t3) == std::vector<uint64_t>{5}));
    // map limit: tickets 6 (map 0) and 7, 8 (map 2) with at most one map
    auto t4 = p.next_tick(8, 1000, 1);
    CHECK((tickets(t4) == std::vector<uint64_t>{6}));
    auto t5 = p.next_tick(8, 1000, 1);
    CHECK((tickets(t5) == std::vector<uint64_t>{7, 8}));
    CHECK(p.queued() == 0 && !p.has_work());
    std::puts("tick formation ok");
}

static void replay_after_full_pool() {
    Planner p(1 << 20);
    int id;
    p.admit(1, &id);
    p.admit(1, &id);
    std::vector<Request> R(6);
    const int maps[6] = {0, 1, 0, 1, 0, 1};
    for (int i = 0; i < 6; ++i) {
        R[i].ticket = (uint64_t)i + 1;
        R[i].map = maps[i];
        R[i].points = 1;
    }
    for (int i = 0; i < 4; ++i) p.submit(&R[i]);
    auto t1 = p.next_tick(2, 100, 8);   // 1 (map 0), 2 (map 1)
    auto t2 = p.next_tick(2, 100, 8);   // 3 (map 0), 4 (map 1)
    p.submit(&R[4]);
    p.submit(&R[5]);
    std::vector<Request*> fin;
    // map 0 is full in tick 1: its request waits for a replay, map 1's completes
    p.complete(t1, {vbx_sched::kPoolFull, 0}, 1.0, &fin);
    CHECK((tickets(fin) == std::vector<uint64_t>{2}));
    CHECK(p.map(0).failed && p.recoverable().empty());   // tick 2 still holds map 0
    // while map 0 waits, only map 1's queued request can run
    auto t3 = p.next_tick(8, 100, 8);
    CHECK((tickets(t3) == std::vector<uint64_t>{6}));
    // tick 2 finds map 0 still in error (the error is sticky until recovery)
    p.complete(t2, {vbx_sched::kPoolFull, 0}, 2.0, &fin);
    CHECK((p.recoverable() == std::vector<int>{0}));
    CHECK((tickets(p.map(0).replay) == std::vector<uint64_t>{1, 3}));
    p.requeue(0);
    auto t4 = p.next_tick(8, 100, 8);
    CHECK((tickets(t4) == std::vector<uint64_t>{1, 3, 5}));
    CHECK(R[0].attempts == 2 && R[4].attempts == 1);
    p.complete(t3, {0}, 3.0, &fin);
    p.complete(t4, {0, 0, 0}, 4.0, &fin);
    CHECK(fin.size() == 6);
    for (const Request& r : R) CHECK(r.state == 2 && r.status == 0);
    // a map that cannot grow runs its turned-away requests one at a time: only the one that
    // overflows on its own fails, the others and later ones are applied in order
    Request a, b, c, d;
    a.ticket = 7; a.map = 0; a.points = 1;
    b.ticket = 8; b.map = 0; b.points = 1;
    c.ticket = 9; c.map = 0; c.points = 1;
    d.ticket = 10; d.map = 0; d.points = 1;
    p.submit(&a);
    p.submit(&b);
    p.submit(&c);
    auto t5 = p.next_tick(8, 100, 8);
    CHECK((tickets(t5) == std::vector<uint64_t>{7, 8, 9}));
    p.submit(&d);
    fin.clear();
    p.complete(t5, {vbx_sched::kPoolFull, vbx_sched::kPoolFull, vbx_sched::kPoolFull}, 5.0, &fin);
    CHECK(fin.empty() && !p.has_work() && (p.recoverable() == std::vector<int>{0}));
    p.requeue(0, true);                                  // no growth: solo replay
    auto t6 = p.next_tick(8, 100, 8);
    CHECK((tickets(t6) == std::vector<uint64_t>{7}) && a.solo);
    CHECK(p.next_tick(8, 100, 8).empty());               // one solo request in flight at a time
    p.complete(t6, {0}, 6.0, &fin);
    auto t7 = p.next_tick(8, 100, 8);
    CHECK((tickets(t7) == std::vector<uint64_t>{8}) && b.solo);
    p.complete(t7, {vbx_sched::kPoolFull}, 7.0, &fin);   // b overflows alone: it fails
    CHECK(b.state == 2 && b.status == vbx_sched::kPoolFull && fin.size() == 2);
    CHECK((p.recoverable() == std::vector<int>{0}) && p.map(0).replay.empty());
    p.requeue(0, true);                                  // error cleared, nothing to replay
    auto t8 = p.next_tick(8, 100, 8);
    CHECK((tickets(t8) == std::vector<uint64_t>{9}) && c.solo);
    p.complete(t8, {0}, 8.0, &fin);
    auto t9 = p.next_tick(8, 100, 8);                    // solo mode is over: d runs normally
    CHECK((tickets(t9) == std::vector<uint64_t>{10}) && !d.solo);
    p.complete(t9, {0}, 9.0, &fin);
    CHECK(a.status == 0 && c.status == 0 && d.status == 0 && fin.size() == 4);
    std::puts("replay ok");
}

// Fake executor: every map has a block capacity; a request adds blocks.  A tick applies its
// requests map by map, in order; a map whose blocks would exceed its capacity is left as it
// was before the tick and reports a full pool, and keeps reporting it (sticky) until the
// scheduler recovers it: by doubling the capacity up to `cap_limit`, else by clearing the
// error and replaying one request at a time.  With up to three ticks in flight, every
// request must end applied exactly once or failed, per-map order must hold among the
// applied ones, and a request may fail only by overflowing the pool alone.
static void simulation(unsigned seed, uint64_t cap_limit) {
    std::mt19937 rng(seed);
    const int M = 12, N = 3000;
    Planner p(1ull << 40);
    std::vector<uint64_t> cap(M), blocks(M, 0);
    std::vector<bool> err(M, false);
    std::vector<std::vector<uint64_t>> applied(M), expect(M);
    for (int m = 0; m < M; ++m) {
        int id;
        cap[(size_t)m] = 8 + rng() % 32;
        CHECK(p.admit(cap[(size_t)m], &id) && id == m);
    }
    std::vector<Request> R(N);
    std::vector<uint64_t> adds(N);
    std::deque<std::vector<Request*>> inflight;
    int next = 0;
    uint64_t done = 0, failed = 0;
    double t = 0.0;
    while (done < (uint64_t)N) {
        const int k = (int)(rng() % 6);
        for (int i = 0; i < k && next < N; ++i, ++next) {
            R[(size_t)next].ticket = (uint64_t)next + 1;
            R[(size_t)next].map = (int)(rng() % M);
            R[(size_t)next].points = 1 + rng() % 50;
            adds[(size_t)next] = rng() % 7 == 0 ? 20 + rng() % 60 : rng() % 5;
            p.submit(&R[(size_t)next]);
        }
        for (int m : p.recoverable()) {
            CHECK(p.map(m).inflight == 0);
            const bool can_grow = !p.map(m).replay.empty() && cap[(size_t)m] * 2 <= cap_limit;
            if (can_grow) cap[(size_t)m] *= 2;
            err[(size_t)m] = false;
            p.requeue(m, !can_grow);
        }
        if (inflight.size() < 3 && p.has_work()) {
            inflight.push_back(p.next_tick(1 + rng() % 16, 200, 5));
            CHECK(!inflight.back().empty());      // has_work promises a non-empty tick
        } else if (inflight.size() < 3) {
            CHECK(p.next_tick(16, 200, 5).empty());
        }
        if (!inflight.empty() && (rng() % 2 == 0 || next == N)) {
            std::vector<Request*> tk = inflight.front();
            inflight.pop_front();
            std::vector<int> status(tk.size(), 0);
            std::map<int, uint64_t> need;
            std::map<int, int> count;
            for (Request* r : tk) {
                need[r->map] += adds[(size_t)(r->ticket - 1)];
                count[r->map]++;
            }
            for (auto& kv : need) {
                const int m = kv.first;
                if (err[(size_t)m] || blocks[(size_t)m] + kv.second > cap[(size_t)m]) err[(size_t)m] = true;
            }
            for (size_t i = 0; i < tk.size(); ++i) {
                const int m = tk[i]->map;
                if (tk[i]->solo) CHECK(count[m] == 1);
                if (err[(size_t)m]) status[i] = vbx_sched::kPoolFull;
                else applied[(size_t)m].push_back(tk[i]->ticket);
            }
            for (auto& kv : need)
                if (!err[(size_t)kv.first]) blocks[(size_t)kv.first] += kv.second;
            std::vector<Request*> fin;
            t += 1.0;
            p.complete(tk, status, t, &fin);
            for (Request* r : fin) {
                if (r->status != 0) {
                    // failed only when run alone, and only by overflowing on its own
                    CHECK(r->status == vbx_sched::kPoolFull && r->solo);
                    CHECK(blocks[(size_t)r->map] + adds[(size_t)(r->ticket - 1)] > cap[(size_t)r->map]);
                    failed++;
                } else {
                    expect[(size_t)r->map].push_back(r->ticket);
                }
            }
            done += fin.size();
        }
    }
    for (int m = 0; m < M; ++m) {
        std::vector<uint64_t> e = expect[(size_t)m];
        std::sort(e.begin(), e.end());
        CHECK(applied[(size_t)m] == e);          // applied once each, in ticket order
    }
    if (cap_limit >= (1ull << 20)) CHECK(failed == 0);
    std::printf("simulation seed %u limit %llu ok (%llu failed)\n", seed, (unsigned long long)cap_limit,
                (unsigned long long)failed);
}

int main() {
    admission();
    tick_formation();
    replay_after_full_pool();
    for (unsigned s = 1; s <= 10; ++s) simulation(s, 1ull << 30);
    for (unsigned s = 11; s <= 20; ++s) simulation(s, 64);
    std::puts("ALL OK");
    return 0;
}
