// Host check of the tile work plans of one launch per level: the level
// kernel's tile remap (for many tile grids and plane counts, the grid of one
// level launch covers every tile of every plane exactly once) and the
// batched level kernel's plan (dwt2_batch_plan.h).
#include <cstdio>
#include <cstdlib>
#include <vector>
#include <cstdint>
#include <algorithm>
#include <random>
#include "dwt2_batch_plan.h"
using namespace dwt2;
// Batched forward, one launch per level: on random batches of uneven
// images, every tile of every image at every level is covered exactly once
// by the per-level grids (with the batched level kernel's XCD remap), the
// work tables fit below the LL area, and every intermediate LL band read or
// written stays inside its own ping-pong buffer.
int run(const std::vector<int>& H, const std::vector<int>& W, int levels, int cx, int core, size_t es) {
    int count = H.size(); int bad = 0;
    LevelBatchLayout L = level_batch_layout(count, levels);
    std::vector<uint32_t> off((size_t)levels * (count + 1));
    for (int l = 0; l < levels; ++l) {
        uint32_t c = 0;
        for (int i = 0; i < count; ++i) { off[l*(count+1)+i] = c; c += (uint32_t)level_tile_count(H[i], W[i], l, cx, core); }
        off[l*(count+1)+count] = c;
    }
    size_t llsum = 0; std::vector<size_t> llo(count);
    for (int i = 0; i < count; ++i) { llo[i] = llsum; llsum += pingpong_ll_bytes(H[i], W[i], levels, es); }
    // tables inside workspace before LL area
    if (L.off_tile + sizeof(uint32_t)*off.size() > L.off_ll_off) bad++;
    if (L.off_ll_off + 8*(size_t)count > L.off_ll) bad++;
    for (int l = 0; l < levels; ++l) {
        uint32_t total = off[l*(count+1)+count];
        const uint32_t chunks = (total + kLevelChunk - 1) / kLevelChunk;
        const uint32_t grid = (chunks + 7) / 8 * 8 * kLevelChunk;
        std::vector<std::vector<int>> seen(count);
        for (int i = 0; i < count; ++i) seen[i].assign(level_tile_count(H[i], W[i], l, cx, core), 0);
        for (uint32_t b = 0; b < grid; ++b) {
            const uint32_t j = b >> 3;
            const uint32_t t = ((j / kLevelChunk) * 8 + (b & 7)) * kLevelChunk + j % kLevelChunk;
            if (t >= total) continue;
            const uint32_t* o = &off[l*(count+1)];
            int lo = 0, hi = count;
            while (hi - lo > 1) { int mid = (lo+hi)>>1; if (o[mid] <= t) lo = mid; else hi = mid; }
            int tt = t - o[lo];
            if (tt < 0 || tt >= (int)seen[lo].size()) { bad++; continue; }
            seen[lo][tt]++;
            // buffer bounds: in / out_ll of this level inside the LL area
            int32_t hl, wl; level_size(H[lo], W[lo], l, &hl, &wl);
            size_t A = llo[lo], B = A + pingpong_b_offset(H[lo], W[lo], levels, es);
            size_t endimg = llo[lo] + pingpong_ll_bytes(H[lo], W[lo], levels, es);
            if (l > 0) {  // input: hl rows of wl elements at pitch ll_pitch(wl)
                size_t base = (l-1)%2==0 ? A : B;
                size_t lastend = base + ((size_t)(hl-1)*ll_pitch(wl) + wl) * es;
                if (lastend > endimg || (((l-1)%2==0) && lastend > B)) { printf("in oob l=%d i=%d\n", l, lo); bad++; }
            }
            if (l + 1 < levels) {
                size_t base = l%2==0 ? A : B;
                int32_t ho = (hl+1)/2, wo = (wl+1)/2;
                size_t lastend = base + ((size_t)(ho-1)*ll_pitch(wo) + wo) * es;
                if (lastend > endimg || ((l%2==0) && lastend > B)) { printf("out oob l=%d i=%d\n", l, lo); bad++; }
            }
        }
        for (int i = 0; i < count; ++i) for (int v : seen[i]) if (v != 1) { bad++; break; }
    }
    return bad;
}
// The level kernel's grid and tile remap (chunks of kRemapRows tile rows
// dealt over 8 XCDs, the tiles of a plane batch taken as one list) cover
// every tile of every plane exactly once.
int check_level_mapping() {
    int bad = 0;
    for (int planes : {1, 2, 3, 5, 17})
        for (int tiles_x = 1; tiles_x <= 40; tiles_x += 3)
            for (int tiles_y = 1; tiles_y <= 700; tiles_y += 7) {
                const int64_t chunk = (int64_t)kRemapRows * tiles_x;
                const int nt = tiles_x * tiles_y;
                const int64_t grid = ((int64_t)nt * planes + 8 * chunk - 1) / (8 * chunk) * (8 * chunk);
                std::vector<int> seen((size_t)nt * planes, 0);
                for (int64_t b = 0; b < grid; ++b) {
                    const int j = (int)(b >> 3);
                    const int g = (int)(((j / chunk) * 8 + (b & 7)) * chunk + j % chunk);
                    if (g < 0) { bad++; continue; }
                    if (g >= nt * planes) continue;
                    const int pl = g / nt, t = g - pl * nt;
                    seen[(size_t)pl * nt + t]++;
                }
                for (int v : seen) if (v != 1) { bad++; break; }
            }
    return bad;
}
int main() {
    if (int b = check_level_mapping()) { printf("level mapping bad %d\n", b); return 1; }
    std::mt19937 rng(7); int bad = 0, cases = 0;
    const int shapes[][2] = {{128, 12}, {128, 28}, {256, 12}, {128, 20}};
    for (const auto& sh : shapes) for (size_t es : {2, 4}) for (int rep = 0; rep < 150; ++rep) {
        const int cx = sh[0], core = sh[1];
        int count = 1 + rng() % 300; std::vector<int> H(count), W(count);
        int lo = 2 + rng() % 64, hi = lo + rng() % 3000;
        for (int i = 0; i < count; ++i) { H[i] = lo + rng() % (hi - lo + 1); W[i] = lo + rng() % (hi - lo + 1); }
        // largest level count for which every transformed level is at least 2 x 2
        int ml = 30;
        for (int i = 0; i < count; ++i) {
            int m = 0; int32_t hl, wl;
            for (;;) { level_size(H[i], W[i], m, &hl, &wl); if (hl < 2 || wl < 2) break; ++m; }
            ml = std::min(ml, m);
        }
        if (ml < 1) continue;
        int levels = 1 + rng() % ml;
        bad += run(H, W, levels, cx, core, es); ++cases;
    }
    printf("cases %d bad %d\n", cases, bad);
    return bad != 0;
}
