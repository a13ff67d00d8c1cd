// Host check of the brick geometry (paper_2103_08932_amd/csrc/bricks.hpp), compiled with g++ against
// the mock HIP header: on random cell grids (empty cells included) of 2D and 3D bodies, for brick
// lengths 1..5 and 8 and the column and tiled brick orders,
//   * brick_coords visits every brick of the grid exactly once, and xcd_block maps the padded grid
//     onto every brick index exactly once;
//   * brick_runs returns, run after run, exactly the particles of the brick's neighbourhood (the
//     cells within one cell of the brick, clipped to the grid) found here by walking the cells, the
//     brick's own particles as [own0, own1), and a first run at offset zero;
//   * a run record written by store_runs and read back by brick_runs_of gives the same runs.
// Exit status 0 and "bricks ok" on success; the first mismatch is printed and ends the run.
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "bricks.hpp"

using namespace tlsph;

#define CHECK(c, ...)                                                     \
    do {                                                                  \
        if (!(c)) {                                                       \
            std::printf("FAIL %s:%d: %s: ", __FILE__, __LINE__, #c);      \
            std::printf(__VA_ARGS__);                                     \
            std::printf("\n");                                            \
            std::exit(1);                                                 \
        }                                                                 \
    } while (0)

template <int D>
static void check_grid(const int nc[3], int zb, const int tile[3], std::mt19937 &rng)
{
    BrickGeom g{};
    g.dim = D;
    for (int k = 0; k < 3; ++k) g.nc[k] = nc[k];
    if (D == 2) g.nc[2] = 1;
    g.zb = zb;
    const int nf = D == 3 ? nc[2] : nc[1];
    g.nbf = (nf + zb - 1) / zb;
    for (int k = 0; k < 3; ++k) g.tile[k] = D == 3 ? tile[k] : 0;
    g.cmap = nullptr;
    g.cmap_words = 0;
    g.runs = nullptr;
    const int64_t ncell = D == 3 ? (int64_t)nc[0] * nc[1] * nc[2] : (int64_t)nc[0] * nc[1];
    // 0..5 particles per cell, three eighths of the cells empty
    std::vector<int32_t> cs(ncell + 1, 0);
    std::uniform_int_distribution<int> cnt(0, 7);
    for (int64_t c = 0; c < ncell; ++c) {
        const int k = cnt(rng);
        cs[c + 1] = cs[c] + (k >= 6 ? 0 : k);
    }
    auto cell = [&](int x, int y, int z) -> int64_t {
        return D == 3 ? ((int64_t)x * nc[1] + y) * nc[2] + z : (int64_t)x * nc[1] + y;
    };
    const int ny = D == 3 ? nc[1] : 1;
    const int64_t nb = brick_count(g);
    CHECK(nb == (int64_t)nc[0] * ny * g.nbf, "brick count %lld", (long long)nb);
    std::vector<int> seen((size_t)nb, 0);
    constexpr int NR = BrickRuns<D>::NR;
    std::vector<int32_t> rec((size_t)nb * run_words<D>(), -7);
    for (int64_t b = 0; b < nb; ++b) {
        int cx, cy, f0;
        brick_coords(g, b, cx, cy, f0);
        if (D == 2) {   // 2D bricks are (cx, fast-axis start); the passes call brick_runs with cy = 0
            CHECK(cy == 0, "2D brick %lld has cy %d", (long long)b, cy);
        }
        CHECK(cx >= 0 && cx < nc[0] && cy >= 0 && cy < ny && f0 >= 0 && f0 < nf && f0 % zb == 0,
              "brick %lld -> (%d, %d, %d) outside the grid", (long long)b, cx, cy, f0);
        const int64_t key = ((int64_t)cx * ny + cy) * g.nbf + f0 / zb;
        CHECK(seen[key] == 0, "brick (%d, %d, %d) visited twice", cx, cy, f0);
        seen[key] = 1;
        BrickRuns<D> R;
        brick_runs<D>(g, cs.data(), cx, cy, f0, R);
        // the neighbourhood by walking its cells: slow-axis offsets ascending, fast axis ascending
        std::vector<int32_t> want;
        for (int r = 0; r < NR; ++r) {
            const int x = D == 3 ? cx + r / 3 - 1 : cx + r - 1;
            const int y = D == 3 ? cy + r % 3 - 1 : 0;
            if (x < 0 || x >= nc[0] || y < 0 || y >= ny) continue;
            for (int f = f0 - 1; f <= f0 + zb; ++f) {
                if (f < 0 || f >= nf) continue;
                const int64_t c = D == 3 ? cell(x, y, f) : cell(x, f, 0);
                for (int32_t j = cs[c]; j < cs[c + 1]; ++j) want.push_back(j);
            }
        }
        std::vector<int32_t> got;
        for (int r = 0; r < NR; ++r)
            for (int k = 0; k < R.len[r]; ++k) got.push_back(R.start[r] + k);
        CHECK(got == want, "brick (%d, %d, %d): %zu particles in its runs, %zu in its cells", cx, cy, f0,
              got.size(), want.size());
        CHECK(R.off[0] == 0 && R.total == (int)want.size(), "brick %lld: off[0] %d total %d", (long long)b,
              R.off[0], R.total);
        for (int r = 0; r + 1 < NR; ++r) CHECK(R.off[r + 1] == R.off[r] + R.len[r], "run offsets of %lld", (long long)b);
        for (int idx = 0; idx < R.total; ++idx)
            CHECK(halo_particle<D>(R, idx) == want[idx], "halo_particle(%d) of brick %lld", idx, (long long)b);
        const int fe = f0 + zb - 1 < nf ? f0 + zb - 1 : nf - 1;
        const int64_t c0 = D == 3 ? cell(cx, cy, f0) : cell(cx, f0, 0);
        const int64_t c1 = D == 3 ? cell(cx, cy, fe) : cell(cx, fe, 0);
        CHECK(R.own0 == cs[c0] && R.own1 == cs[c1 + 1], "own range of brick %lld", (long long)b);
        // the run record round trip
        store_runs<D>(R, rec.data() + b * run_words<D>());
    }
    for (int64_t k = 0; k < nb; ++k) CHECK(seen[k] == 1, "brick %lld never visited", (long long)k);
    g.runs = rec.data();
    for (int64_t b = 0; b < nb; ++b) {
        int cx, cy, f0;
        brick_coords(g, b, cx, cy, f0);
        BrickRuns<D> R, Q;
        brick_runs<D>(g, cs.data(), cx, cy, f0, R);
        brick_runs_of<D>(g, b, Q);
        bool same = R.total == Q.total && R.own0 == Q.own0 && R.own1 == Q.own1;
        for (int r = 0; r < NR; ++r)
            same = same && R.start[r] == Q.start[r] && R.off[r] == Q.off[r] && R.len[r] == Q.len[r];
        CHECK(same, "record of brick %lld differs from its runs", (long long)b);
    }
    // XCD remap: every brick index exactly once over the padded grid
    std::vector<int> hit((size_t)nb, 0);
    const int64_t ng = xcd_grid(nb);
    CHECK(ng % kXcds == 0 && ng >= nb && ng < nb + kXcds, "xcd_grid(%lld) = %lld", (long long)nb, (long long)ng);
    for (int64_t w = 0; w < ng; ++w) {
        const int64_t l = xcd_block(w, nb);
        if (l < 0) continue;
        CHECK(l < nb && hit[l] == 0, "xcd_block(%lld) = %lld", (long long)w, (long long)l);
        hit[l] = 1;
    }
    for (int64_t k = 0; k < nb; ++k) CHECK(hit[k] == 1, "brick %lld not launched", (long long)k);
}

int main()
{
    std::mt19937 rng(20240521u);
    const int grids3[][3] = {{1, 1, 1}, {3, 2, 7}, {5, 4, 11}, {9, 6, 17}, {2, 9, 4}};
    const int tiles[][3] = {{0, 0, 0}, {4, 4, 16}, {2, 3, 2}, {1, 1, 1}, {3, 5, 7}};
    const int zbs[] = {1, 2, 3, 4, 5, 8};
    int cases = 0;
    for (const auto &nc : grids3)
        for (const auto &t : tiles)
            for (int zb : zbs) {
                check_grid<3>(nc, zb, t, rng);
                ++cases;
            }
    const int grids2[][3] = {{1, 1, 1}, {7, 13, 1}, {4, 3, 1}, {12, 25, 1}};
    const int none[3] = {0, 0, 0};
    for (const auto &nc : grids2)
        for (int zb : zbs) {
            check_grid<2>(nc, zb, none, rng);
            ++cases;
        }
    std::printf("bricks ok: %d geometries\n", cases);
    return 0;
}
