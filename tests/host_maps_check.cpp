// Host-side checks of index maps the kernels use (compiled by hipcc as a
// host program by tests/test_host_maps.py; no device code runs).
#include <cstdio>
#include <vector>

#include "../paper_1310_7866_amd/csrc/psc_internal.h"
#include "../paper_1310_7866_amd/csrc/psc_xcd.h"

using namespace psc;

static int failures = 0;
#define CHECK(cond, ...)                         \
    do {                                         \
        if (!(cond)) {                           \
            std::printf("FAIL: " __VA_ARGS__);   \
            std::printf("\n");                   \
            ++failures;                          \
        }                                        \
    } while (0)

// The mixed-lane ablation: over the rounds of a work item (workgroups of nt
// lanes, lane g = r0 + thread), every strip [0, nruns) is taken by exactly
// one lane and no lane takes a strip outside it.
static void check_mix_lane() {
    for (int nt : {256, 384, 512})
        for (int nruns = 0; nruns <= 3000; ++nruns) {
            std::vector<int> seen(nruns, 0);
            for (int r0 = 0; r0 < nruns; r0 += nt)
                for (int t = 0; t < nt; ++t) {
                    const int g = mix_lane(r0 + t, nruns);
                    CHECK(g >= 0 && g <= 64 * ((nruns + 63) / 64), "mix_lane(%d, %d) = %d out of range", r0 + t, nruns, g);
                    if (g >= 0 && g < nruns) ++seen[g];
                }
            for (int g = 0; g < nruns; ++g)
                CHECK(seen[g] == 1, "nt %d nruns %d: strip %d taken %d times", nt, nruns, g, seen[g]);
        }
}

// The particle kernel's key of a cell just outside a patch: equals the
// general encoder of the wrapped geometric cell, for every patch and every
// local coordinate within one cell of it, on grids with truncated last
// patches, single patches along a dimension, and 2-d (x invariant) runs.
static void check_neighbour_key() {
    struct G { int n[3], P[3]; };
    const G grids[] = {{{1, 12, 9}, {1, 4, 4}}, {{1, 10, 7}, {1, 4, 3}}, {{1, 8, 5}, {1, 8, 2}},
                       {{7, 9, 6}, {3, 4, 2}}, {{8, 8, 8}, {4, 4, 4}}, {{5, 6, 7}, {5, 2, 3}},
                       {{9, 4, 10}, {4, 4, 3}}};
    for (const G &g : grids) {
        RunDev r{};
        for (int d = 0; d < 3; ++d) {
            r.n[d] = g.n[d];
            r.P[d] = g.P[d];
            r.np[d] = (g.n[d] + g.P[d] - 1) / g.P[d];
        }
        r.dim = g.n[0] == 1 ? 2 : 3;
        for (int p = 0; p < r.np[0] * r.np[1] * r.np[2]; ++p) {
            int pc[3];
            patch_coords(r, p, pc);
            const int h[3] = {patch_ext(r, 0, pc[0]), patch_ext(r, 1, pc[1]), patch_ext(r, 2, pc[2])};
            const int lo0 = r.dim == 2 ? 0 : -1, hi0 = r.dim == 2 ? 0 : h[0];
            for (int a = lo0; a <= hi0; ++a)
                for (int b = -1; b <= h[1]; ++b)
                    for (int c = -1; c <= h[2]; ++c) {
                        const int l[3] = {a, b, c};
                        const int gi = wrap(pc[0] * r.P[0] + a, r.n[0]), gj = wrap(pc[1] * r.P[1] + b, r.n[1]),
                                  gk = wrap(pc[2] * r.P[2] + c, r.n[2]);
                        const int64_t want = encode_key(r, gi, gj, gk), got = neighbour_key(r, pc, h, l);
                        CHECK(want == got, "grid %dx%dx%d patch %d local (%d,%d,%d): %lld != %lld", r.n[0], r.n[1],
                              r.n[2], p, a, b, c, (long long)got, (long long)want);
                    }
        }
    }
}

// The direct current path: for every geometry current_direct_fits accepts
// (cells n, patch P, order), every tile coordinate of every patch maps by
// wrap_near onto the same cell as the general periodic wrap, inside [0, n)
// (and the test covers refused geometries too).
static void check_current_direct_map() {
    int accepted = 0, refused = 0;
    for (int order = 1; order <= 2; ++order)
        for (int n = 1; n <= 40; ++n)
            for (int P = 1; P <= 48; ++P) {
                const int lo = cur_lo(order), hi = cur_hi(order), jt = P + lo + hi;
                const int np = (n + P - 1) / P;
                bool in_range = true;
                for (int pc = 0; pc < np; ++pc)
                    for (int t = 0; t < jt; ++t) {
                        const int i = pc * P + t - lo;
                        const int w = wrap_near(i, n);
                        in_range &= w >= 0 && w < n && w == wrap(i, n);
                    }
                if (current_direct_fits(n, P, order)) {
                    ++accepted;
                    CHECK(in_range, "order %d n %d P %d: a tile coordinate leaves [0, n)", order, n, P);
                } else {
                    ++refused;
                }
            }
    CHECK(accepted > 0 && refused > 0, "direct-path geometries: %d accepted, %d refused", accepted, refused);
}

// The sort's closed-form order of the source cells of a new cell (one move
// against each move code) equals the order of their keys, found by brute
// force, for every cell of grids with truncated last patches, single
// patches and 3-cell axes, in 2-d and 3-d; and the ranks are 0 .. M - 1.
template <int DIM>
static void check_source_ranks_grid(const int n[3], const int P[3]) {
    constexpr int M = DIM == 3 ? 27 : 9;
    RunDev r{};
    r.dim = DIM;
    for (int d = 0; d < 3; ++d) {
        r.n[d] = n[d];
        r.P[d] = P[d];
        r.np[d] = (n[d] + P[d] - 1) / P[d];
    }
    const int64_t nc = (int64_t)n[0] * n[1] * n[2];
    for (int64_t key = 0; key < nc; ++key) {
        int g[3], pc[3], l[3];
        decode_key(r, key, g);
        Axis ax[3];
        for (int d = 0; d < 3; ++d) {
            pc[d] = g[d] / P[d];
            l[d] = g[d] - pc[d] * P[d];
            ax[d] = axis_neighbours(P[d], n[d], r.np[d], pc[d], l[d]);
        }
        int rk[M];
        source_ranks<DIM>(ax, rk);
        uint32_t ks[M];
        for (int m = 0; m < M; ++m) {
            int dm[3];
            move_delta(DIM, m, dm);
            const int a0 = DIM == 3 ? 1 - dm[0] : 1, a1 = 1 - dm[1], a2 = 1 - dm[2];
            ks[m] = key_of(r, ax[0].pc[a0], ax[1].pc[a1], ax[2].pc[a2], ax[0].l[a0], ax[1].l[a1], ax[2].l[a2],
                           ax[0].ext[a0], ax[1].ext[a1], ax[2].ext[a2]);
            // the source is the wrapped cell one move back
            const int gi = wrap(g[0] - dm[0], n[0]), gj = wrap(g[1] - dm[1], n[1]), gk = wrap(g[2] - dm[2], n[2]);
            CHECK((int64_t)ks[m] == encode_key(r, gi, gj, gk), "grid %dx%dx%d key %lld move %d: wrong source",
                  n[0], n[1], n[2], (long long)key, m);
        }
        int seen[M] = {0};
        for (int m = 0; m < M; ++m) {
            int want = 0;
            for (int q = 0; q < M; ++q) want += ks[q] < ks[m] ? 1 : 0;
            CHECK(rk[m] == want, "grid %dx%dx%d patch %dx%dx%d key %lld move %d: rank %d, key order %d", n[0], n[1],
                  n[2], P[0], P[1], P[2], (long long)key, m, rk[m], want);
            if (rk[m] >= 0 && rk[m] < M) ++seen[rk[m]];
        }
        for (int k = 0; k < M; ++k) CHECK(seen[k] == 1, "key %lld: rank %d taken %d times", (long long)key, k, seen[k]);
    }
}

static void check_source_ranks() {
    struct G { int n[3], P[3]; };
    const G g3[] = {{{8, 8, 8}, {4, 4, 4}}, {{10, 9, 7}, {4, 4, 4}}, {{7, 9, 6}, {3, 4, 2}}, {{3, 3, 3}, {3, 3, 3}},
                    {{5, 6, 7}, {5, 2, 3}}, {{9, 4, 10}, {4, 4, 3}}, {{16, 16, 20}, {8, 8, 8}}, {{3, 5, 4}, {1, 2, 4}}};
    for (const G &g : g3) check_source_ranks_grid<3>(g.n, g.P);
    const G g2[] = {{{1, 12, 9}, {1, 4, 4}}, {{1, 10, 7}, {1, 4, 3}}, {{1, 8, 5}, {1, 8, 2}}, {{1, 3, 3}, {1, 3, 3}},
                    {{1, 20, 12}, {1, 8, 8}}, {{1, 18, 12}, {1, 8, 8}}, {{1, 5, 9}, {1, 1, 4}}};
    for (const G &g : g2) check_source_ranks_grid<2>(g.n, g.P);
}

// The XCD placement of workgroups: a bijection on [0, G) for every grid size,
// and the workgroups one XCD runs (b = x, x + 8, ...) map onto one contiguous
// range in order.
static void check_xcd_map() {
    for (uint32_t G = 1; G <= 3000; ++G) {
        std::vector<int> seen(G, 0);
        for (uint32_t b = 0; b < G; ++b) {
            const uint32_t L = xcd_map(b, G);
            CHECK(L < G, "xcd_map(%u, %u) = %u out of range", b, G, L);
            if (L < G) ++seen[L];
            if (b >= kXcds) CHECK(L == xcd_map(b - kXcds, G) + 1, "G %u: workgroup %u not after %u", G, b, b - kXcds);
        }
        for (uint32_t L = 0; L < G; ++L) CHECK(seen[L] == 1, "G %u: index %u taken %d times", G, L, seen[L]);
    }
}

int main() {
    check_xcd_map();
    check_mix_lane();
    check_neighbour_key();
    check_current_direct_map();
    check_source_ranks();
    if (failures) {
        std::printf("%d failures\n", failures);
        return 1;
    }
    std::printf("ok\n");
    return 0;
}
