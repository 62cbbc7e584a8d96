// Host-side planning of the all-pairs work (see dd_host.h); plain C++.
#include "dd_host.h"

#include <algorithm>
#include <cmath>

namespace dd {

// Source-range length of a work item when none is given: at least about 2048
// work items; source ranges of at least MIN_CHUNK_LEN sources (small problems
// spread over many CUs), in whole TILEs above that, and no longer than
// max(512, N_max / 16): the largest items set the tail of the schedule, and
// splitting them further costs only partial sums (on many bursts or one very
// large volume this is 7-12 % faster than one range per tile).
int64_t heuristic_chunk(int64_t total_tiles, int64_t max_src)
{
    const int64_t want_items = 2048, MIN_CHUNK = MIN_CHUNK_LEN;
    int64_t chunks = total_tiles > 0 ? (want_items + total_tiles - 1) / total_tiles : 1;
    chunks = std::max<int64_t>(1, std::min<int64_t>(chunks, (max_src + MIN_CHUNK - 1) / MIN_CHUNK));
    int64_t chunk_len = (max_src + chunks - 1) / chunks;
    chunk_len = std::min<int64_t>(chunk_len, std::max<int64_t>(512, (max_src + 15) / 16));
    const int64_t gran = chunk_len > TILE ? TILE : MIN_CHUNK;
    return std::max<int64_t>(MIN_CHUNK, (chunk_len + gran - 1) / gran * gran);
}

// chunk_len <= 0: choose so that a single large volume fills the chip.
void make_plan(const std::vector<int64_t> &seg_off, int Q, int64_t chunk_len, Plan &P,
               const std::vector<uint8_t> *active)
{
    const int n_inst = (int)seg_off.size() - 1;
    P.tiles.clear();
    P.items.clear();
    P.tile_begin.assign(n_inst + 1, 0);
    if (chunk_len <= 0) {
        int64_t total_tiles = 0, max_src = 0;
        for (int i = 0; i < n_inst; ++i) {
            if (active && !(*active)[i]) continue;
            int64_t N = seg_off[i + 1] - seg_off[i];
            total_tiles += (N * Q + TILE - 1) / TILE;
            max_src = std::max(max_src, N);
        }
        chunk_len = heuristic_chunk(total_tiles, max_src);
    }
    P.chunk_len = chunk_len;
    int64_t slot = 0;
    for (int i = 0; i < n_inst; ++i) {
        const int64_t s0 = seg_off[i], N = seg_off[i + 1] - s0;
        P.tile_begin[i] = (int64_t)P.tiles.size();
        if (active && !(*active)[i]) continue;   // an idle instance gets no tiles
        const int64_t npts = N * Q;
        const int nchunks = N > 0 ? (int)((N + chunk_len - 1) / chunk_len) : 0;
        for (int64_t pb = 0; pb < npts; pb += TILE) {
            Tile t;
            t.point_begin = s0 * Q + pb;
            t.n_points = (int32_t)std::min<int64_t>(TILE, npts - pb);
            t.n_chunks = nchunks;
            t.slot_begin = slot;
            const int32_t tidx = (int32_t)P.tiles.size();
            P.tiles.push_back(t);
            for (int c = 0; c < nchunks; ++c) {
                Item it;
                it.tile = tidx;
                it.pad = 0;
                it.src_begin = s0 + c * chunk_len;
                it.src_end = std::min(s0 + N, it.src_begin + chunk_len);
                it.slot = slot++;
                P.items.push_back(it);
            }
        }
    }
    P.tile_begin[n_inst] = (int64_t)P.tiles.size();
    // longest items first: the dispatcher hands out workgroups in index order,
    // which makes this a longest-processing-time-first schedule
    std::stable_sort(P.items.begin(), P.items.end(), [&](const Item &a, const Item &b) {
        const int64_t ca = (int64_t)P.tiles[a.tile].n_points * (a.src_end - a.src_begin);
        const int64_t cb = (int64_t)P.tiles[b.tile].n_points * (b.src_end - b.src_begin);
        return ca > cb;
    });
}

// Gauss-Legendre rule on [0, 1]: the roots z of P_n are found by Newton's
// method on the Legendre recurrence (k P_k = (2k-1) z P_{k-1} - (k-1) P_{k-2})
// from the guess cos(pi (4i + 3) / (4n + 2)); P_n'(z) = n (z P_n - P_{n-1}) /
// (z^2 - 1) and the weight on [-1, 1] is 2 / ((1 - z^2) P_n'(z)^2).
GaussRule gauss_rule(int n)
{
    GaussRule g{};
    g.n = n;
    for (int i = 0; i < n; ++i) {
        double z = std::cos(3.14159265358979323846 * (4.0 * i + 3.0) / (4.0 * n + 2.0));
        double p = 0, q = 0, dp = 1;
        for (int it = 0; it < 60; ++it) {
            q = 1.0;   // P_{k-1}
            p = z;     // P_k
            for (int k = 2; k <= n; ++k) {
                double r = ((2 * k - 1) * z * p - (k - 1) * q) / k;
                q = p;
                p = r;
            }
            dp = n * (z * p - q) / (z * z - 1.0);
            double step = p / dp;
            z -= step;
            if (std::fabs(step) < 1e-17) break;
        }
        q = 1.0; p = z;
        for (int k = 2; k <= n; ++k) {
            double r = ((2 * k - 1) * z * p - (k - 1) * q) / k;
            q = p;
            p = r;
        }
        dp = n * (z * p - q) / (z * z - 1.0);
        // i = 0 is the largest root
        g.s[n - 1 - i] = 0.5 * (1.0 + z);
        g.w[n - 1 - i] = 1.0 / ((1.0 - z * z) * dp * dp);
    }
    return g;
}

}  // namespace dd
