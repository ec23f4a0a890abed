// Randomised check of the server arena's first-fit bookkeeping (host only):
// ranges never overlap and stay inside the arena, the used count matches the
// live ranges, free ranges stay merged, and everything returns to one range.
#include "../paper_1201_5651_amd/csrc/arena.h"

#include <cstdio>
#include <random>
#include <vector>

int main()
{
    pi::ArenaMap m;
    const size_t size = 1 << 20;
    m.init(size + 100);   // rounded down to 256-byte granules
    if (m.size != size) return 1;
    std::mt19937_64 rng(5651);
    struct Live { size_t off, n; };
    std::vector<Live> live;
    for (int it = 0; it < 200000; ++it) {
        if (live.empty() || rng() % 3 != 0) {
            const size_t n = 1 + rng() % 40000;
            size_t off;
            if (m.alloc(n, &off)) {
                const size_t r = pi::ArenaMap::round(n);
                if (off % 256 || off + r > size) return 2;
                for (const Live& l : live)
                    if (off < l.off + l.n && l.off < off + r) return 3;
                live.push_back({ off, r });
            } else {
                // first fit fails only when no free range is large enough
                for (auto& f : m.free_)
                    if (f.second >= pi::ArenaMap::round(n)) return 4;
            }
        } else {
            const size_t k = rng() % live.size();
            m.release(live[k].off, live[k].n);
            live.erase(live.begin() + k);
        }
        size_t used = 0;
        for (const Live& l : live) used += l.n;
        if (used != m.used) return 5;
        size_t prev_end = (size_t)-1, freed = 0;
        for (auto& f : m.free_) {
            if (f.first == prev_end) return 6;   // adjacent free ranges not merged
            prev_end = f.first + f.second;
            freed += f.second;
        }
        if (freed + used != size) return 7;
    }
    for (const Live& l : live) m.release(l.off, l.n);
    if (m.used != 0 || m.free_.size() != 1 || m.free_.begin()->second != size) return 8;
    std::printf("arena ok\n");
    return 0;
}
