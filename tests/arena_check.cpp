// Host test driver for the server's arena allocator (no HIP): a random
// sequence of allocations and releases checked against a brute-force model
// of the occupied bytes.  Prints "ok" and exits 0 on success.
#include <stdio.h>
#include <stdlib.h>

#include <random>
#include <vector>

#include "../paper_1406_6158_amd/csrc/arena.h"

using htree::Arena;

static int fail(const char *what, long a, long b) {
    printf("FAIL %s %ld %ld\n", what, a, b);
    return 1;
}

int main() {
    const size_t size = 1 << 20;
    Arena A(size + 100);    // rounded down to the alignment
    if (A.size() != size) return fail("size", (long)A.size(), (long)size);
    std::vector<char> busy(size / Arena::kAlign, 0);
    struct Blk { size_t off, bytes; };
    std::vector<Blk> live;
    std::mt19937_64 rng(7);
    for (int it = 0; it < 200000; it++) {
        bool do_alloc = live.empty() || (rng() % 100) < 55;
        if (do_alloc) {
            size_t want = 1 + rng() % (size / 16);
            size_t off = A.alloc(want);
            size_t need = Arena::round_up(want) / Arena::kAlign;
            // is there a free run of `need` units?  first fit must match the lowest
            size_t run = 0, first = Arena::kNone;
            for (size_t u = 0; u < busy.size(); u++) {
                run = busy[u] ? 0 : run + 1;
                if (run == need) { first = (u + 1 - need) * Arena::kAlign; break; }
            }
            if (off != first) return fail("first fit", (long)off, (long)first);
            if (off == Arena::kNone) continue;
            if (off % Arena::kAlign) return fail("alignment", (long)off, 0);
            for (size_t u = off / Arena::kAlign; u < off / Arena::kAlign + need; u++) busy[u] = 1;
            live.push_back({off, need * Arena::kAlign});
        } else {
            size_t k = rng() % live.size();
            if (!A.release(live[k].off)) return fail("release", (long)live[k].off, 0);
            if (A.release(live[k].off)) return fail("double release", (long)live[k].off, 0);
            for (size_t u = live[k].off / Arena::kAlign;
                 u < (live[k].off + live[k].bytes) / Arena::kAlign; u++)
                busy[u] = 0;
            live[k] = live.back();
            live.pop_back();
        }
        size_t used = 0;
        for (char b : busy) used += b;
        if (A.used() != used * Arena::kAlign) return fail("used", (long)A.used(), (long)used);
        if (A.live_blocks() != live.size()) return fail("live", (long)A.live_blocks(), (long)live.size());
        if (it % 1000 == 0) {
            // free blocks are maximal runs: their count equals the number of free runs
            size_t runs = 0;
            for (size_t u = 0; u < busy.size(); u++)
                if (!busy[u] && (u == 0 || busy[u - 1])) runs++;
            if (A.free_blocks() != runs) return fail("coalesce", (long)A.free_blocks(), (long)runs);
        }
    }
    for (auto &b : live) A.release(b.off);
    if (A.used() != 0 || A.free_blocks() != 1 || A.largest_free() != size)
        return fail("drain", (long)A.used(), (long)A.free_blocks());
    if (A.alloc(size + 1) != Arena::kNone) return fail("oversize", 0, 0);
    if (A.alloc(size) != 0) return fail("whole", 0, 0);
    printf("ok\n");
    return 0;
}
