// Host scheduling core of the map server: admission of maps under a device-memory budget,
// per-map FIFO order of integration requests, formation of the next batch ("tick") for
// continuous batching, and the replay of requests that a full block pool turned away.
//
// Free of device code and of locking (the server holds its lock around every call), so it
// can be exercised with a plain host compiler.
#pragma once

#include <algorithm>
#include <cstdint>
#include <deque>
#include <vector>

namespace vbx_sched {

// Status values shared with the C ABI.
constexpr int kOk = 0;
constexpr int kPoolFull = -3;

struct Request {
    uint64_t ticket = 0;      // submission order, from 1
    int map = -1;
    uint64_t points = 0;
    double t_arrival = 0.0;   // seconds on the server clock
    double t_done = 0.0;
    int status = kOk;
    int state = 0;            // 0 queued, 1 in a tick, 2 finished
    int attempts = 0;         // ticks this request was part of
    bool solo = false;        // last taken as its map's only request, nothing of it in flight
};

struct MapSlot {
    uint64_t bytes = 0;             // device memory charged to the budget
    int inflight = 0;               // ticks in flight holding requests of this map
    bool failed = false;            // a tick found the map's pool full: awaiting recovery
    std::vector<Request*> replay;   // requests to run again once recovered, ticket order
    uint64_t solo = 0;              // next requests of the map that must run one at a time
};

class Planner {
public:
    explicit Planner(uint64_t budget) : budget_(budget) {}

    uint64_t budget() const { return budget_; }
    uint64_t used() const { return used_; }
    int num_maps() const { return (int)maps_.size(); }
    const MapSlot& map(int id) const { return maps_[(size_t)id]; }
    size_t queued() const { return queue_.size(); }

    // Admits a map that needs `bytes` of device memory; false (nothing charged) when the
    // budget cannot hold it.
    bool admit(uint64_t bytes, int* id) {
        if (bytes > budget_ - used_) return false;
        used_ += bytes;
        maps_.emplace_back();
        maps_.back().bytes = bytes;
        *id = (int)maps_.size() - 1;
        return true;
    }

    // Charges `extra` bytes for the growth of map `id`; false when over budget.
    bool grow(int id, uint64_t extra) {
        if (extra > budget_ - used_) return false;
        used_ += extra;
        maps_[(size_t)id].bytes += extra;
        return true;
    }

    // Returns bytes charged by grow() that were not used.
    void release(int id, uint64_t bytes) {
        MapSlot& m = maps_[(size_t)id];
        bytes = std::min(bytes, m.bytes);
        m.bytes -= bytes;
        used_ -= bytes;
    }

    // Appends a request; tickets must increase.
    void submit(Request* r) {
        r->state = 0;
        queue_.push_back(r);
    }

    // True exactly when next_tick would return something: some queued request's map neither
    // awaits recovery nor is in solo mode with a tick in flight (the first queued request of
    // such a map is always taken by an empty tick).
    bool has_work() const {
        for (const Request* r : queue_)
            if (eligible(maps_[(size_t)r->map])) return true;
        return false;
    }

    // The next tick: queued requests in ticket order, passing over maps that await recovery
    // (a map's requests run in ticket order, so all of its queued requests wait), until
    // adding one more would exceed max_frames, max_points or max_maps distinct maps.  A
    // request larger than max_points on its own forms a tick by itself.  A map in solo mode
    // contributes one request, and only when none of its ticks is in flight.
    std::vector<Request*> next_tick(size_t max_frames, uint64_t max_points, size_t max_maps) {
        std::vector<Request*> tick;
        std::vector<int> seen, held;
        std::deque<Request*> rest;
        uint64_t pts = 0;
        bool closed = false;
        for (Request* r : queue_) {
            MapSlot& m = maps_[(size_t)r->map];
            const bool new_map = std::find(seen.begin(), seen.end(), r->map) == seen.end();
            const bool hold = !eligible(m) || std::find(held.begin(), held.end(), r->map) != held.end() ||
                              (m.solo > 0 && !new_map);
            if (closed || hold) {
                if (!closed && !m.failed) held.push_back(r->map);   // keeps the map's order
                rest.push_back(r);
                continue;
            }
            if (!tick.empty() && (tick.size() >= max_frames || pts + r->points > max_points ||
                                  (new_map && seen.size() >= max_maps))) {
                closed = true;
                rest.push_back(r);
                continue;
            }
            tick.push_back(r);
            pts += r->points;
            r->solo = m.solo > 0;
            if (r->solo) {
                m.solo--;
                held.push_back(r->map);   // the map's only request in this tick
            }
            if (new_map) {
                seen.push_back(r->map);
                m.inflight++;
            }
        }
        queue_.swap(rest);
        for (Request* r : tick) {
            r->state = 1;
            r->attempts++;
        }
        return tick;
    }

    // A tick has completed at time t.  map_status[i] is the status its call left on the map
    // of tick[i].  Requests of a map whose pool was full go to that map's replay list (the
    // map is unchanged by them), except a request that ran solo: it alone overflowed the
    // pool and finishes with that status.  The others finish with their status.  Finished
    // requests are appended to *finished.
    void complete(const std::vector<Request*>& tick, const std::vector<int>& map_status, double t,
                  std::vector<Request*>* finished) {
        std::vector<int> seen;
        for (size_t i = 0; i < tick.size(); ++i) {
            Request* r = tick[i];
            MapSlot& m = maps_[(size_t)r->map];
            if (std::find(seen.begin(), seen.end(), r->map) == seen.end()) {
                seen.push_back(r->map);
                m.inflight--;
            }
            if (map_status[i] == kPoolFull && r->solo) {
                m.failed = true;          // the map's error is cleared before it runs again
                r->status = kPoolFull;
                r->t_done = t;
                r->state = 2;
                finished->push_back(r);
            } else if (map_status[i] == kPoolFull) {
                m.failed = true;
                r->state = 0;
                auto it = std::lower_bound(m.replay.begin(), m.replay.end(), r,
                                           [](const Request* a, const Request* b) { return a->ticket < b->ticket; });
                m.replay.insert(it, r);
            } else {
                r->status = map_status[i];
                r->t_done = t;
                r->state = 2;
                finished->push_back(r);
            }
        }
    }

    // Maps that wait for recovery with no tick of theirs in flight.
    std::vector<int> recoverable() const {
        std::vector<int> out;
        for (size_t i = 0; i < maps_.size(); ++i)
            if (maps_[i].failed && maps_[i].inflight == 0) out.push_back((int)i);
        return out;
    }

    // After map `id` has room again (or had its error cleared): its replay requests go back
    // into the queue ahead of its later requests (ticket order overall).  With `solo`, they
    // run one per tick, so that each one that still overflows the pool fails on its own.
    void requeue(int id, bool solo = false) {
        MapSlot& m = maps_[(size_t)id];
        if (solo) m.solo += m.replay.size();
        for (Request* r : m.replay) {
            auto it = std::lower_bound(queue_.begin(), queue_.end(), r,
                                       [](const Request* a, const Request* b) { return a->ticket < b->ticket; });
            queue_.insert(it, r);
        }
        m.replay.clear();
        m.failed = false;
    }

private:
    static bool eligible(const MapSlot& m) { return !m.failed && !(m.solo > 0 && m.inflight > 0); }

    uint64_t budget_;
    uint64_t used_ = 0;
    std::vector<MapSlot> maps_;
    std::deque<Request*> queue_;   // ticket order
};

}  // namespace vbx_sched
