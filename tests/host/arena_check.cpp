// Host-side checks of the serving arena (paper_2304_12745_amd/csrc/server_arena.h),
// built with AddressSanitizer and UndefinedBehaviorSanitizer by
// tests/test_server_host.py.  Exit status 0 = every check passed.
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "../../paper_2304_12745_amd/csrc/server_arena.h"

using dmimo::Arena;
using dmimo::align256;

static int failures = 0;
#define CHECK(c)                                                        \
    do {                                                                \
        if (!(c)) {                                                     \
            std::fprintf(stderr, "check failed line %d: %s\n", __LINE__, #c); \
            ++failures;                                                 \
        }                                                               \
    } while (0)

struct Block {
    size_t off, bytes;
};

// free list: disjoint, coalesced, inside the arena; used blocks disjoint from
// it and from each other; free + used = size
static void check_invariants(const Arena& a, const std::vector<Block>& used) {
    size_t end = 0, total = 0;
    bool first = true;
    for (const auto& kv : a.free_list()) {
        CHECK(kv.second > 0 && kv.first % 256 == 0 && kv.second % 256 == 0);
        if (!first) CHECK(kv.first > end);   // disjoint and never adjacent (coalesced)
        end = kv.first + kv.second;
        CHECK(end <= a.size());
        total += kv.second;
        first = false;
    }
    size_t u = 0;
    for (size_t i = 0; i < used.size(); ++i) {
        const Block& b = used[i];
        u += align256(b.bytes);
        CHECK(b.off + align256(b.bytes) <= a.size());
        for (const auto& kv : a.free_list())
            CHECK(b.off + align256(b.bytes) <= kv.first || kv.first + kv.second <= b.off);
        for (size_t j = i + 1; j < used.size(); ++j) {
            const Block& c = used[j];
            CHECK(b.off + align256(b.bytes) <= c.off || c.off + align256(c.bytes) <= b.off);
        }
    }
    CHECK(total + u == a.size());
}

int main() {
    // 1. geometry uploaded between running queries: with resident data at the
    //    top, the freed query space is one block again, and a query that fills
    //    everything below the resident data is admitted
    {
        Arena a;
        const size_t size = 64 << 20;
        a.init(size);
        std::vector<Block> used;
        size_t q1, q2, g1, q3;
        CHECK(a.alloc_low(10 << 20, &q1));
        used.push_back({q1, 10 << 20});
        CHECK(a.alloc_high(3 << 20, &g1));   // add_deployment while q1 runs
        used.push_back({g1, 3 << 20});
        CHECK(g1 == size - (3 << 20));
        CHECK(a.alloc_low(20 << 20, &q2));
        used.push_back({q2, 20 << 20});
        check_invariants(a, used);
        a.release(q1, 10 << 20);
        a.release(q2, 20 << 20);
        used = {{g1, 3 << 20}};
        check_invariants(a, used);
        CHECK(a.blocks() == 1 && a.largest_free() == size - (3 << 20));
        CHECK(a.alloc_low(size - (3 << 20), &q3));   // the whole space below the geometry
        CHECK(q3 == 0);
        used.push_back({q3, size - (3 << 20)});
        check_invariants(a, used);
        size_t x;
        CHECK(!a.alloc_low(256, &x) && !a.alloc_high(256, &x));
    }
    // 2. random interleaving of query scratch (alloc_low / release) and
    //    resident uploads (alloc_high, never released), with the invariants
    //    after every operation and the one-block property whenever no query
    //    holds memory
    {
        std::mt19937_64 rng(12345);
        for (int round = 0; round < 50; ++round) {
            Arena a;
            const size_t size = (size_t)(1 + rng() % 256) << 20 | (rng() % 4096);   // not a multiple of 256
            a.init(size);
            CHECK(a.size() == (size & ~size_t(255)));
            std::vector<Block> q, res;
            for (int op = 0; op < 400; ++op) {
                const int kind = (int)(rng() % 10);
                if (kind < 5) {
                    const size_t bytes = 1 + rng() % (a.size() / 8 + 1);
                    size_t off;
                    if (a.alloc_low(bytes, &off)) q.push_back({off, bytes});
                } else if (kind < 9) {
                    if (!q.empty()) {
                        const size_t i = rng() % q.size();
                        a.release(q[i].off, q[i].bytes);
                        q.erase(q.begin() + (long)i);
                    }
                } else {
                    const size_t bytes = 1 + rng() % (a.size() / 32 + 1);
                    size_t off;
                    if (a.alloc_high(bytes, &off)) res.push_back({off, bytes});
                }
                std::vector<Block> all = q;
                all.insert(all.end(), res.begin(), res.end());
                check_invariants(a, all);
                // the resident blocks form one stack at the top
                size_t lowest_res = a.size(), res_bytes = 0;
                for (const Block& b : res) {
                    lowest_res = b.off < lowest_res ? b.off : lowest_res;
                    res_bytes += align256(b.bytes);
                }
                CHECK(lowest_res == a.resident_floor());
                CHECK(a.size() - lowest_res == res_bytes);
                for (const Block& b : q) CHECK(b.off + align256(b.bytes) <= lowest_res);
                if (q.empty() && a.free_bytes() > 0) {
                    // no query holds memory: the free space is one block below the stack
                    CHECK(a.blocks() == 1);
                    CHECK(a.free_list().begin()->first == 0);
                    CHECK(a.largest_free() == lowest_res);
                }
            }
        }
    }
    // 3. exact fits, zero-byte requests and full release
    {
        Arena a;
        a.init(4096);
        size_t o1, o2, o3;
        CHECK(a.alloc_low(0, &o1) && o1 == 0);          // rounds up to one 256-byte block
        CHECK(a.alloc_high(256, &o2) && o2 == 4096 - 256);
        CHECK(a.alloc_low(4096 - 512, &o3) && o3 == 256);
        size_t x;
        CHECK(!a.alloc_low(1, &x));
        a.release(o3, 4096 - 512);
        a.release(o1, 0);
        a.release(o2, 256);
        CHECK(a.blocks() == 1 && a.free_bytes() == 4096);
    }
    if (failures) {
        std::fprintf(stderr, "%d checks failed\n", failures);
        return 1;
    }
    std::printf("arena checks passed\n");
    return 0;
}
