// Host replay of the persistent forward transform's work queue, built on the
// library's plan header (dwt2_batch_plan.h): the planner's tables computed
// as the planner kernel computes them, then one thread per work-group
// running the persistent kernel's loop (ticket from the lowest level with
// tickets, own sub-queue first; the image of the ticket, by bisection here,
// which finds the same image as the kernel's 64-way search; tile of the
// ticket; wait for the chunks of the previous level; publish).  The
// "computation" of a tile checks, by brute force and independently of
// dep_chunks, that every tile of the previous level whose LL rows the tile
// reads (its input rows with the halo, reflected at the image edges) has
// finished, then marks the tile.  Checked on random batches and plane
// stacks for every tile shape: no wait runs out, every tile of every level
// of every image runs exactly once, every read is of a finished tile, and
// the tables and LL bands stay inside the workspace.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstdint>
#include <cstdio>
#include <random>
#include <thread>
#include <vector>

#include "dwt2_batch_plan.h"

using namespace dwt2;

namespace {

struct Img { int h, w; };

int check(const std::vector<Img>& im, int levels, int cx, int cy, int grid, size_t es) {
    const int count = (int)im.size();
    int bad = 0;
    // planner tables
    std::vector<uint32_t> coff((size_t)levels * (count + 1)), qoff((size_t)levels * kXcds * (count + 1)),
        cbase(levels + 1);
    uint32_t base = 0;
    uint64_t tiles_total = 0;
    for (int l = 0; l < levels; ++l) {
        uint32_t c = 0, q[kXcds] = {};
        for (int i = 0; i < count; ++i) {
            int32_t hl, wl, tx, ty;
            level_size(im[i].h, im[i].w, l, &hl, &wl);
            level_tiles(hl, wl, cx, cy, &tx, &ty);
            coff[(size_t)l * (count + 1) + i] = c;
            uint32_t sum = 0;
            for (int y = 0; y < kXcds; ++y) {
                qoff[((size_t)l * kXcds + y) * (count + 1) + i] = q[y];
                const uint32_t n = subqueue_tiles(c, y, tx, ty);
                q[y] += n;
                sum += n;
            }
            if (sum != (uint32_t)tx * (uint32_t)ty) { printf("subqueue tiles %u != %d\n", sum, tx * ty); ++bad; }
            tiles_total += (uint64_t)tx * ty;
            c += (uint32_t)chunk_count(ty);
        }
        coff[(size_t)l * (count + 1) + count] = c;
        for (int y = 0; y < kXcds; ++y) qoff[((size_t)l * kXcds + y) * (count + 1) + count] = q[y];
        cbase[l] = base;
        base += c;
    }
    cbase[levels] = base;
    // workspace layout
    const BatchLayout L = batch_layout(count, levels, base);
    size_t ll = 0;
    std::vector<size_t> ll_off(count);
    for (int i = 0; i < count; ++i) { ll_off[i] = ll; ll += image_ll_bytes(im[i].h, im[i].w, levels, es); }
    if (!(kHeaderBytes <= L.off_taken && L.off_taken + 4 * kCounterStride * levels * kXcds <= L.off_coff &&
          L.off_coff + 4 * coff.size() <= L.off_qoff && L.off_qoff + 4 * qoff.size() <= L.off_cbase &&
          L.off_cbase + 4 * cbase.size() <= L.off_ll_off && L.off_ll_off % 8 == 0 &&
          L.off_ll_off + 8 * (size_t)count <= L.off_done && L.off_done + 4 * (size_t)base <= L.off_ll &&
          L.off_ll % 256 == 0)) { printf("layout\n"); ++bad; }
    // LL bands: level l's band holds (h_l+1)/2 rows at pitch ll_pitch((w_l+1)/2), inside the image's bands
    for (int i = 0; i < count; ++i)
        for (int l = 0; l + 1 < levels; ++l) {
            int32_t hl, wl;
            level_size(im[i].h, im[i].w, l, &hl, &wl);
            const size_t o = ll_band_offset(im[i].h, im[i].w, l, es);
            const size_t end = o + ((size_t)((hl + 1) / 2 - 1) * ll_pitch((wl + 1) / 2) + (wl + 1) / 2) * es;
            if (o % 256 || end > ll_band_offset(im[i].h, im[i].w, l + 1, es) ||
                end > image_ll_bytes(im[i].h, im[i].w, levels, es)) { printf("band\n"); ++bad; }
        }
    // tile state per (level, image)
    std::vector<std::vector<std::atomic<int>>> st((size_t)levels * count);
    std::vector<int> TX((size_t)levels * count), TY((size_t)levels * count), HL((size_t)levels * count);
    for (int l = 0; l < levels; ++l)
        for (int i = 0; i < count; ++i) {
            int32_t hl, wl, tx, ty;
            level_size(im[i].h, im[i].w, l, &hl, &wl);
            level_tiles(hl, wl, cx, cy, &tx, &ty);
            const size_t k = (size_t)l * count + i;
            TX[k] = tx; TY[k] = ty; HL[k] = hl;
            st[k] = std::vector<std::atomic<int>>((size_t)tx * ty);
            for (auto& s : st[k]) s.store(0);
        }
    std::vector<std::atomic<uint32_t>> taken((size_t)levels * kXcds), done(base);
    for (auto& t : taken) t.store(0);
    for (auto& d : done) d.store(0);
    std::atomic<long> timeouts{0}, violations{0}, twice{0}, oob{0};
    auto work = [&](int b) {
        const int home = b & (kXcds - 1);
        int lvl = 0;
        uint32_t empty = 0;
        for (;;) {
            int tl = -1, ty = 0;
            uint32_t tp = 0;
            while (lvl < levels && tl < 0) {
                for (int k = 0; k < kXcds; ++k) {
                    const int y = (home + k) & (kXcds - 1);
                    if (empty & (1u << y)) continue;
                    const uint32_t n = qoff[((size_t)lvl * kXcds + y) * (count + 1) + count];
                    const uint32_t p = n ? taken[(size_t)lvl * kXcds + y].fetch_add(1) : 0u;
                    if (p < n) { tl = lvl; ty = y; tp = p; break; }
                    empty |= 1u << y;
                }
                if (tl < 0) { ++lvl; empty = 0; }
            }
            if (tl < 0) return;
            const int l = tl, y = ty;
            const uint32_t* q = &qoff[((size_t)l * kXcds + y) * (count + 1)];
            int lo = 0, hi = count;
            while (hi - lo > 1) { const int mid = (lo + hi) >> 1; if (q[mid] <= tp) lo = mid; else hi = mid; }
            const int i = lo;
            const size_t k = (size_t)l * count + i;
            const uint32_t g0 = coff[(size_t)l * (count + 1) + i];
            int32_t row, col, chunk;
            subqueue_tile(g0, y, TX[k], tp - q[i], &row, &col, &chunk);
            if (row < 0 || row >= TY[k] || col < 0 || col >= TX[k] || chunk >= chunk_count(TY[k])) { ++oob; continue; }
            if (l > 0) {
                const size_t kp = (size_t)(l - 1) * count + i;
                int32_t c0, c1;
                dep_chunks(row, cy, HL[k], &c0, &c1);
                const uint32_t db = cbase[l - 1] + coff[(size_t)(l - 1) * (count + 1) + i];
                // bounded as in the kernel (here 2 s of wall-clock time per tile)
                const auto t0 = std::chrono::steady_clock::now();
                for (int32_t c = c1; c >= c0; --c)
                    while (done[db + c].load(std::memory_order_acquire) < chunk_tiles(c, TX[kp], TY[kp])) {
                        if (std::chrono::steady_clock::now() - t0 > std::chrono::seconds(2)) { ++timeouts; break; }
                        std::this_thread::yield();
                    }
                // brute force: every input row of the tile (core rows and halo, reflected at the edges)
                const int hl = HL[k];
                for (int64_t r = 2 * ((int64_t)row * cy - kHalo); r < 2 * ((int64_t)(row + 1) * cy + kHalo); ++r) {
                    int64_t rr = r;
                    while (rr < 0 || rr >= hl) rr = rr < 0 ? -rr : 2 * (hl - 1) - rr;   // whole-point symmetric
                    const int trow = (int)(rr / cy);                                    // LL row rr of level l-1
                    for (int c = 0; c < TX[kp]; ++c)
                        if (st[kp][(size_t)trow * TX[kp] + c].load() != 1) { ++violations; break; }
                }
            }
            if (st[k][(size_t)row * TX[k] + col].fetch_add(1) != 0) ++twice;
            done[cbase[l] + g0 + chunk].fetch_add(1, std::memory_order_release);
        }
    };
    std::vector<std::thread> th;
    for (int b = 0; b < grid; ++b) th.emplace_back(work, b);
    for (auto& t : th) t.join();
    long missing = 0;
    for (auto& v : st) for (auto& s : v) if (s.load() != 1) ++missing;
    for (int l = 0; l < levels; ++l)
        for (int i = 0; i < count; ++i) {
            const size_t k = (size_t)l * count + i;
            for (int c = 0; c < chunk_count(TY[k]); ++c)
                if (done[cbase[l] + coff[(size_t)l * (count + 1) + i] + c].load() != chunk_tiles(c, TX[k], TY[k])) ++bad;
        }
    bad += (int)(timeouts + violations + twice + oob + missing);
    if (bad) printf("count %d levels %d tile %dx%d grid %d: timeouts %ld violations %ld twice %ld oob %ld missing %ld\n",
                    count, levels, cx, cy, grid, timeouts.load(), violations.load(), twice.load(), oob.load(), missing);
    return bad;
}

int max_levels(int h, int w) {
    int n = 0;
    while (h >= 2 && w >= 2) { ++n; h = (h + 1) / 2; w = (w + 1) / 2; }
    return n;
}

}  // namespace

// dep_chunks against brute force, independent of timing: every chunk of
// level l-1 holding a row that a tile of level l loads (its rows with the
// halo, reflected at the edges) lies in the range dep_chunks gives.
int check_dep_chunks() {
    int bad = 0;
    for (int cy : {12, 20, 28})
        for (int hl = 2; hl < 2500; ++hl) {
            const int ty = ((hl + 1) / 2 + cy - 1) / cy;
            for (int row = 0; row < ty; ++row) {
                int32_t c0, c1;
                dep_chunks(row, cy, hl, &c0, &c1);
                for (int64_t r = 2 * ((int64_t)row * cy - kHalo); r < 2 * ((int64_t)(row + 1) * cy + kHalo); ++r) {
                    int64_t rr = r;
                    while (rr < 0 || rr >= hl) rr = rr < 0 ? -rr : 2 * (hl - 1) - rr;
                    const int c = (int)(rr / cy) / kChunkRows;
                    if (c < c0 || c > c1) { ++bad; break; }
                }
            }
        }
    return bad;
}

int main() {
    std::mt19937 rng(11);
    int bad = check_dep_chunks(), cases = 0;
    if (bad) printf("dep_chunks misses rows in %d tiles\n", bad);
    // (core columns, core rows) of the tile configurations
    const int shapes[][2] = {{128, 12}, {128, 28}, {256, 12}, {128, 20}};
    for (const auto& sh : shapes)
        for (int rep = 0; rep < 40; ++rep) {
            const bool stack = rep % 4 == 3;
            int count = stack ? 1 + rng() % 12 : 1 + rng() % 60;
            const int lo = 2 + rng() % 40, hi = lo + rng() % (rep % 5 == 0 ? 9000 : 1500);
            std::vector<Img> im(count);
            for (int i = 0; i < count; ++i) {
                im[i] = {lo + (int)(rng() % (hi - lo + 1)), lo + (int)(rng() % (hi - lo + 1))};
                if (stack) im[i] = im[0];
            }
            int ml = 40;
            for (auto& x : im) ml = std::min(ml, max_levels(x.h, x.w));
            if (ml < 1) continue;
            const int levels = 1 + rng() % ml;
            const int grids[] = {8, 24, 64, 200};
            bad += check(im, levels, sh[0], sh[1], grids[rng() % 4], rep % 2 ? 2 : 4);
            ++cases;
        }
    // the benchmark's shapes: one 8192^2 image at 5 levels, 64 planes of 256^2
    bad += check({{8192, 8192}}, 5, 128, 20, 64, 4);
    bad += check(std::vector<Img>(64, {256, 256}), 5, 128, 20, 64, 4);
    cases += 2;
    printf("cases %d bad %d\n", cases, bad);
    return bad != 0;
}
