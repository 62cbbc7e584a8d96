// Host planning code (paper_2005_02498_amd/csrc/dd_host.cpp) under
// AddressSanitizer and UBSan: builds work plans for many instance layouts and
// checks their invariants, and checks the Gauss-Legendre rules against exact
// polynomial integrals.  Prints "<k> failures" and exits 0 only when k = 0.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <random>
#include <set>
#include <vector>

#include "dd_host.h"

using namespace dd;

static int failures = 0;
#define CHECK(c, ...)                                        \
    do {                                                     \
        if (!(c)) {                                          \
            ++failures;                                      \
            std::printf("FAIL %s:%d: ", __FILE__, __LINE__); \
            std::printf(__VA_ARGS__);                        \
            std::printf("\n");                               \
        }                                                    \
    } while (0)

// Every target point of an active instance is in exactly one tile; every
// (tile, source of its instance) pair in exactly one item; slots are unique
// and each tile's items use slot_begin .. slot_begin + n_chunks - 1; items are
// sorted by cost, longest first; idle instances get no tiles.
static void check_plan(const std::vector<int64_t> &off, int Q, int64_t chunk, const std::vector<uint8_t> *act)
{
    Plan P;
    make_plan(off, Q, chunk, P, act);
    const int n = (int)off.size() - 1;
    CHECK((int)P.tile_begin.size() == n + 1, "tile_begin size");
    CHECK(P.chunk_len >= MIN_CHUNK_LEN || (chunk > 0 && P.chunk_len == chunk), "chunk_len %lld",
          (long long)P.chunk_len);
    std::set<int64_t> slots;
    std::vector<std::vector<std::pair<int64_t, int64_t>>> ranges(P.tiles.size());
    for (const Item &it : P.items) {
        CHECK(it.tile >= 0 && it.tile < (int)P.tiles.size(), "item tile %d", it.tile);
        if (it.tile < 0 || it.tile >= (int)P.tiles.size()) continue;
        const Tile &t = P.tiles[it.tile];
        CHECK(it.slot >= t.slot_begin && it.slot < t.slot_begin + t.n_chunks, "slot outside its tile's range");
        CHECK(slots.insert(it.slot).second, "slot %lld used twice", (long long)it.slot);
        CHECK(it.src_begin < it.src_end, "empty source range");
        CHECK(it.src_end - it.src_begin <= P.chunk_len, "source range longer than chunk_len");
        ranges[it.tile].push_back({it.src_begin, it.src_end});
    }
    CHECK((int64_t)slots.size() == (int64_t)P.items.size(), "slot count");
    for (size_t k = 1; k < P.items.size(); ++k) {
        const Item &a = P.items[k - 1], &b = P.items[k];
        const int64_t ca = (int64_t)P.tiles[a.tile].n_points * (a.src_end - a.src_begin);
        const int64_t cb = (int64_t)P.tiles[b.tile].n_points * (b.src_end - b.src_begin);
        CHECK(ca >= cb, "items not sorted longest first");
    }
    for (int i = 0; i < n; ++i) {
        const int64_t s0 = off[i], N = off[i + 1] - off[i];
        const bool on = !act || (*act)[i];
        const int64_t tb = P.tile_begin[i], te = P.tile_begin[i + 1];
        CHECK(tb <= te, "tile_begin not monotonic");
        if (!on || N == 0) {
            CHECK(tb == te, "instance %d (idle or empty) has tiles", i);
            continue;
        }
        int64_t next = s0 * Q;
        for (int64_t k = tb; k < te; ++k) {
            const Tile &t = P.tiles[k];
            CHECK(t.point_begin == next, "instance %d: points not covered in order", i);
            CHECK(t.n_points >= 1 && t.n_points <= TILE, "tile size %d", t.n_points);
            next = t.point_begin + t.n_points;
            auto r = ranges[k];
            std::sort(r.begin(), r.end());
            CHECK((int)r.size() == t.n_chunks, "tile has %zu items, n_chunks %d", r.size(), t.n_chunks);
            int64_t s = s0;
            for (auto &p : r) {
                CHECK(p.first == s, "instance %d: sources not covered exactly once", i);
                s = p.second;
            }
            CHECK(s == s0 + N, "instance %d: sources end at %lld, not %lld", i, (long long)s, (long long)(s0 + N));
        }
        CHECK(next == (s0 + N) * Q, "instance %d: points end early", i);
    }
}

static void check_heuristic()
{
    for (int64_t tiles : {1LL, 3LL, 64LL, 1000LL, 100000LL})
        for (int64_t src : {1LL, 15LL, 16LL, 17LL, 255LL, 4096LL, 262144LL}) {
            const int64_t c = heuristic_chunk(tiles, src);
            CHECK(c >= MIN_CHUNK_LEN, "heuristic_chunk(%lld, %lld) = %lld", (long long)tiles, (long long)src,
                  (long long)c);
            CHECK(c % (c > TILE ? TILE : MIN_CHUNK_LEN) == 0, "heuristic_chunk not a whole granule");
        }
}

// Gauss-Legendre with n points integrates s^k exactly on [0, 1] for k < 2n.
static void check_gauss()
{
    for (int n = 1; n <= DD_MAX_GAUSS; ++n) {
        const GaussRule g = gauss_rule(n);
        CHECK(g.n == n, "rule size");
        for (int i = 0; i < n; ++i) {
            CHECK(g.s[i] > 0.0 && g.s[i] < 1.0 && g.w[i] > 0.0, "n=%d point %d outside (0,1)", n, i);
            if (i) CHECK(g.s[i] > g.s[i - 1], "n=%d points not ascending", n);
            CHECK(std::fabs(g.s[i] + g.s[n - 1 - i] - 1.0) < 1e-14, "n=%d not symmetric", n);
        }
        for (int k = 0; k < 2 * n; ++k) {
            double sum = 0.0;
            for (int i = 0; i < n; ++i) sum += g.w[i] * std::pow(g.s[i], k);
            CHECK(std::fabs(sum - 1.0 / (k + 1)) < 1e-13, "n=%d k=%d: %.17g", n, k, sum);
        }
    }
}

int main()
{
    check_heuristic();
    check_gauss();
    std::mt19937_64 rng(7);
    // hand-picked layouts: one large volume, empty and single-segment
    // instances, sizes around TILE, many small bursts
    std::vector<std::vector<int64_t>> sizes = {
        {16384}, {0}, {1}, {1, 0, 2}, {255, 256, 257}, {128, 128, 128, 128}, {5000, 3, 0, 17}};
    {
        std::vector<int64_t> many;
        for (int i = 0; i < 512; ++i) many.push_back(32 + (int64_t)(rng() % 4064));
        sizes.push_back(many);
    }
    for (int r = 0; r < 40; ++r) {
        std::vector<int64_t> v(1 + rng() % 20);
        for (auto &x : v) x = (int64_t)(rng() % 3000);
        sizes.push_back(v);
    }
    int plans = 0;
    for (const auto &sz : sizes) {
        std::vector<int64_t> off(sz.size() + 1, 0);
        for (size_t i = 0; i < sz.size(); ++i) off[i + 1] = off[i] + sz[i];
        std::vector<uint8_t> act(sz.size());
        for (auto &a : act) a = (uint8_t)(rng() % 3 != 0);
        for (int Q : {1, 2, 3, 4, 16})
            for (int64_t chunk : {0LL, 16LL, 100LL, 512LL, 1024LL, 1LL << 20}) {
                check_plan(off, Q, chunk, nullptr);
                check_plan(off, Q, chunk, &act);
                plans += 2;
            }
    }
    std::printf("%d plans checked, %d failures\n", plans, failures);
    return failures == 0 ? 0 : 1;
}
