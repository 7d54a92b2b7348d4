// CPU test of the request scheduler (serve_core.h) with a fake executor:
// arena allocation, FIFO admission under a memory budget, batch size and
// slot limits, completion and release, launch failures, and a randomized
// simulation checking the invariants at every step.  Prints "OK" on success.
#include <cstdio>
#include <cstdlib>
#include <random>
#include <set>
#include <vector>

#include "serve_core.h"

using namespace kr::serve;

#define CHECK(cond)                                                                   \
    do {                                                                              \
        if (!(cond)) {                                                                \
            std::fprintf(stderr, "FAILED %s:%d: %s\n", __FILE__, __LINE__, #cond);    \
            std::exit(1);                                                             \
        }                                                                             \
    } while (0)

struct FakeExec {
    std::vector<std::vector<Admitted>> running;  // per slot
    std::vector<int> remaining;                  // steps until done
    std::vector<std::vector<uint64_t>> launched_ids;
    int fail_next = 0;
    int delay = 1;
    std::mt19937 *rng = nullptr;
    explicit FakeExec(int slots) : running(slots), remaining(slots, 0) {}
    bool launch(int s, const std::vector<Admitted> &b)
    {
        if (fail_next > 0) {
            fail_next--;
            return false;
        }
        CHECK(running[s].empty());
        running[s] = b;
        remaining[s] = rng ? 1 + (int)((*rng)() % 4) : delay;
        std::vector<uint64_t> ids;
        for (const auto &a : b)
            ids.push_back(a.req.id);
        launched_ids.push_back(ids);
        return true;
    }
    bool done(int s)
    {
        if (running[s].empty())
            return true;
        if (--remaining[s] > 0)
            return false;
        running[s].clear();
        return true;
    }
};

static Request req(uint64_t id, size_t bytes)
{
    Request r;
    r.id = id;
    r.dst_bytes = bytes;
    return r;
}

static void test_arena()
{
    Arena a(4096, 256);
    size_t o1, o2, o3, o4;
    CHECK(a.alloc(100, &o1) && o1 == 0);
    CHECK(a.alloc(256, &o2) && o2 == 256);
    CHECK(a.alloc(1000, &o3) && o3 == 512);
    CHECK(a.used() == 256 + 256 + 1024);
    CHECK(!a.alloc(4096, &o4));
    CHECK(a.release(o2));
    CHECK(!a.release(o2));           // double free is refused
    CHECK(a.alloc(200, &o4) && o4 == 256);  // first fit reuses the hole
    CHECK(a.release(o1) && a.release(o4) && a.release(o3));
    CHECK(a.used() == 0 && a.largest_free() == 4096);  // fully coalesced
    CHECK(a.alloc(4096, &o1) && o1 == 0);
    CHECK(a.release(o1));
    // fragmentation: free every other block, then a large one does not fit
    std::vector<size_t> offs(16);
    for (auto &o : offs)
        CHECK(a.alloc(256, &o));
    for (size_t i = 0; i < offs.size(); i += 2)
        CHECK(a.release(offs[i]));
    CHECK(a.largest_free() == 256);
    CHECK(!a.alloc(512, &o1));
    for (size_t i = 1; i < offs.size(); i += 2)
        CHECK(a.release(offs[i]));
    CHECK(a.largest_free() == 4096);
}

static void test_fifo_budget_and_limits()
{
    FakeExec ex(2);
    ex.delay = 2;
    Scheduler<FakeExec> s(ex, 4096, 2, 3);
    CHECK(!s.submit(req(99, 5000)));  // can never fit
    for (uint64_t i = 0; i < 6; i++)
        CHECK(s.submit(req(i, 1024)));
    std::vector<Completion> out;
    CHECK(s.step(0.0, out));
    // slot 0 takes 3 (batch limit), slot 1 the fourth (budget 4 x 1024 exhausted)
    CHECK(ex.launched_ids.size() == 2);
    CHECK((ex.launched_ids[0] == std::vector<uint64_t>{0, 1, 2}));
    CHECK((ex.launched_ids[1] == std::vector<uint64_t>{3}));
    CHECK(s.arena().used() == 4096 && s.queued() == 2 && s.busy_slots() == 2);
    CHECK(s.step(1.0, out) && out.empty());
    CHECK(s.step(2.0, out));
    CHECK(out.size() == 4);  // both batches done; outputs still held
    CHECK(ex.launched_ids.size() == 2 && s.queued() == 2);  // nothing admitted: memory is full
    for (const auto &c : out)
        CHECK(c.t_done == 2.0);
    CHECK(s.release(out[0].dst_off) && s.release(out[1].dst_off));
    out.clear();
    CHECK(s.step(3.0, out));
    CHECK(ex.launched_ids.size() == 3);
    CHECK((ex.launched_ids[2] == std::vector<uint64_t>{4, 5}));
}

static void test_head_of_line_waits()
{
    FakeExec ex(4);
    Scheduler<FakeExec> s(ex, 4096, 4, 8);
    CHECK(s.submit(req(0, 3000)));
    CHECK(s.submit(req(1, 3000)));  // cannot fit while 0 holds memory
    CHECK(s.submit(req(2, 100)));   // small, but behind 1: must not overtake it
    std::vector<Completion> out;
    CHECK(s.step(0, out));
    CHECK(ex.launched_ids.size() == 1 && ex.launched_ids[0].size() == 1 && s.queued() == 2);
    CHECK(s.step(1, out) && out.size() == 1);
    CHECK(ex.launched_ids.size() == 1);  // 0 done but not released: 1 still waits, 2 too
    CHECK(s.release(out[0].dst_off));
    out.clear();
    CHECK(s.step(2, out));
    CHECK(ex.launched_ids.size() == 2);
    CHECK((ex.launched_ids[1] == std::vector<uint64_t>{1, 2}));
}

static void test_launch_failure_requeues()
{
    FakeExec ex(1);
    Scheduler<FakeExec> s(ex, 4096, 1, 4);
    for (uint64_t i = 0; i < 3; i++)
        CHECK(s.submit(req(i, 512)));
    ex.fail_next = 1;
    std::vector<Completion> out;
    CHECK(!s.step(0, out));
    CHECK(s.queued() == 3 && s.arena().used() == 0 && s.busy_slots() == 0);
    CHECK(s.step(1, out));
    CHECK((ex.launched_ids.back() == std::vector<uint64_t>{0, 1, 2}));
}

// The budget is the server's own memory: the output blocks it allocates.
// Sources are the caller's resident buffers, which the server neither copies
// nor allocates, so their size does not enter admission.
static void test_admission_counts_outputs_only()
{
    FakeExec ex(1);
    Scheduler<FakeExec> s(ex, 4096, 1, 8);
    Request big_src = req(0, 1024);
    big_src.sh = 2160;
    big_src.sw = 3840;  // a 24.9 MB source, far above the 4 KiB budget
    CHECK(s.submit(big_src));
    CHECK(s.submit(req(1, 3072)));
    CHECK(s.submit(req(2, 256)));  // over the budget once 0 and 1 hold it
    std::vector<Completion> out;
    CHECK(s.step(0, out));
    CHECK((ex.launched_ids[0] == std::vector<uint64_t>{0, 1}));
    CHECK(s.arena().used() == 4096 && s.queued() == 1);
}

static void test_random_simulation()
{
    std::mt19937 rng(1234);
    const int slots = 3, max_batch = 5;
    const size_t budget = 1 << 16;
    FakeExec ex(slots);
    ex.rng = &rng;
    Scheduler<FakeExec> s(ex, budget, slots, max_batch);
    const int n = 3000;
    std::set<uint64_t> completed;
    std::vector<std::pair<size_t, int>> held;  // (offset, steps until release)
    uint64_t next = 0, last_admitted = 0;
    bool first = true;
    for (int step = 0; completed.size() < (size_t)n; step++) {
        CHECK(step < 1000000);
        while (next < (uint64_t)n && rng() % 3 == 0)
            CHECK(s.submit(req(next++, 1 + rng() % (budget / 4))));
        std::vector<Completion> out;
        CHECK(s.step((double)step, out));
        for (const auto &c : out) {
            CHECK(completed.insert(c.id).second);  // each request completes once
            held.push_back({c.dst_off, (int)(rng() % 3)});
        }
        for (size_t i = 0; i < held.size();) {
            if (held[i].second-- <= 0) {
                CHECK(s.release(held[i].first));
                held[i] = held.back();
                held.pop_back();
            } else {
                i++;
            }
        }
        CHECK(s.arena().used() <= budget);
        CHECK(s.busy_slots() <= slots);
        // admission order is FIFO across all launches (in launch order)
        for (const auto &ids : ex.launched_ids) {
            CHECK((int)ids.size() <= max_batch);
            for (size_t k = 1; k < ids.size(); k++)
                CHECK(ids[k] == ids[k - 1] + 1);
            CHECK(first || ids.front() == last_admitted + 1);
            last_admitted = ids.back();
            first = false;
        }
        ex.launched_ids.clear();
    }
    CHECK(s.idle());
}

int main()
{
    test_arena();
    test_fifo_budget_and_limits();
    test_head_of_line_waits();
    test_launch_failure_requeues();
    test_admission_counts_outputs_only();
    test_random_simulation();
    std::printf("OK\n");
    return 0;
}
