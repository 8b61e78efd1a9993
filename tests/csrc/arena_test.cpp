// Host-only test of the graph-capture ownership rules (symba_arena.h): the
// capture arena never hands out the same byte twice, respects alignment and
// capacity; the partial-sum buffer is kept, grown, retired or refused as the
// rules say.  Built with g++ (no HIP) by tests/test_arena_host.py.
#include "symba_arena.h"

#include <cstdio>
#include <cstdlib>
#include <vector>

static int failures = 0;
#define CHECK(c)                                                   \
    do {                                                           \
        if (!(c)) {                                                \
            std::printf("FAIL %s:%d: %s\n", __FILE__, __LINE__, #c); \
            ++failures;                                            \
        }                                                          \
    } while (0)

int main() {
    using symba::BumpArena;
    using symba::PartialAction;
    using symba::plan_partial;
    {  // disjoint, aligned, append-only, bounded
        BumpArena a(10000);
        std::vector<std::pair<size_t, size_t>> got;
        size_t off = 0;
        const size_t sizes[] = {608, 1, 2432, 256, 7, 6000, 1, 600};
        for (size_t b : sizes) {
            if (a.alloc(b, 256, off)) got.push_back({off, b});
        }
        for (size_t i = 0; i < got.size(); ++i) {
            CHECK(got[i].first % 256 == 0);
            CHECK(got[i].first + got[i].second <= a.capacity());
            for (size_t j = 0; j < i; ++j)  // later blocks start after every earlier block ends
                CHECK(got[i].first >= got[j].first + got[j].second);
        }
        CHECK(got.size() == 7);  // the 6000-byte block does not fit after the first five; later small ones do
        const size_t used = a.used();
        CHECK(!a.alloc(a.capacity(), 256, off));
        CHECK(a.used() == used);  // a refused request changes nothing
        CHECK(!a.alloc(16, 3, off));  // alignment must be a power of two
        BumpArena z(0);
        CHECK(!z.alloc(1, 1, off));
        CHECK(z.alloc(0, 1, off) && off == 0);
        BumpArena big(~size_t(0));
        CHECK(big.alloc(~size_t(0) - 100, 1, off));
        CHECK(!big.alloc(1, 256, off));  // rounding up would wrap around: refused
    }
    {  // partial-sum buffer
        PartialAction p = plan_partial(1000, 800, false, false);
        CHECK(p.kind == PartialAction::Keep && p.new_bytes == 1000);
        p = plan_partial(1000, 800, true, true);  // fits: fine even under capture
        CHECK(p.kind == PartialAction::Keep);
        p = plan_partial(1000, 1200, false, true);  // would have to allocate under capture
        CHECK(p.kind == PartialAction::Refuse);
        p = plan_partial(1000, 1200, false, false);  // grow; nothing captured uses the old one: free it
        CHECK(p.kind == PartialAction::Grow && p.new_bytes >= 1200 && !p.retire_old);
        CHECK(p.new_bytes == 1500);  // geometric
        p = plan_partial(1000, 5000, true, false);  // a capture uses the old one: retire it
        CHECK(p.kind == PartialAction::Grow && p.new_bytes == 5000 && p.retire_old);
        p = plan_partial(0, 256, false, false);
        CHECK(p.kind == PartialAction::Grow && p.new_bytes == 256 && !p.retire_old);
        // a run of growth retires at most about as much as the final buffer holds
        size_t cur = 256, retired = 0;
        for (size_t need = 300; need < 1000000; need = need * 11 / 10) {
            const PartialAction q = plan_partial(cur, need, true, false);
            if (q.kind == PartialAction::Grow) {
                if (q.retire_old) retired += cur;
                cur = q.new_bytes;
            }
        }
        CHECK(retired <= 3 * cur);
    }
    std::printf(failures ? "failed\n" : "ok\n");
    return failures ? 1 : 0;
}
