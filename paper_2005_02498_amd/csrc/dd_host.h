// Host-side planning of the all-pairs work, in plain C++ (no HIP): the split
// of one force pass into tiles of target Gauss points and work items of
// source ranges, and the Gauss-Legendre rule of the target quadrature.  Built
// by the host compiler into libdd.so, and with AddressSanitizer and UBSan by
// the CPU test suite (tests/asan/host_driver.cpp checks the invariants).
#pragma once

#include <cstdint>
#include <vector>

#include "dd.h"

namespace dd {

constexpr int TILE = 256;          // target Gauss points per tile (one workgroup)
constexpr int MIN_CHUNK_LEN = 16;  // shortest source range of a work item

struct Tile {
    int64_t point_begin;   // global Gauss-point index (segment * Q + q)
    int32_t n_points;      // <= TILE
    int32_t n_chunks;      // items covering this tile, slots slot_begin..+n_chunks
    int64_t slot_begin;
};

struct Item {
    int32_t tile;
    int32_t pad;
    int64_t src_begin;     // global segment indices [src_begin, src_end)
    int64_t src_end;
    int64_t slot;          // partial-sum slot
};

struct GaussRule {
    double s[DD_MAX_GAUSS];
    double w[DD_MAX_GAUSS];
    int n;
};

// Work decomposition for a set of instances (host tables): instance i's
// target points s0 Q .. (s0 + N) Q - 1 (segments s0 = seg_off[i], N of them)
// in tiles of TILE points; each tile paired with every source range of
// chunk_len segments of its own instance as one item with a slot of its own.
// Items are sorted longest first (points x sources).
struct Plan {
    std::vector<Tile> tiles;
    std::vector<Item> items;
    std::vector<int64_t> tile_begin;   // [n_inst+1]
    int64_t chunk_len = 0;
};

// Source-range length of a work item when none is given.
int64_t heuristic_chunk(int64_t total_tiles, int64_t max_src);

// chunk_len <= 0: choose with heuristic_chunk.  active (nullable, [n_inst]):
// instances with 0 get no tiles.
void make_plan(const std::vector<int64_t> &seg_off, int Q, int64_t chunk_len, Plan &P,
               const std::vector<uint8_t> *active = nullptr);

// Gauss-Legendre rule of n points on [0, 1] (1 <= n <= DD_MAX_GAUSS).
GaussRule gauss_rule(int n);

}  // namespace dd
