// Host-side checks of index maps the kernels use (compiled by hipcc as a
// host program by tests/test_host_maps.py; no device code runs).
#include <cstdio>
#include <vector>

#include "../paper_1310_7866_amd/csrc/psc_internal.h"

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

int main() {
    check_mix_lane();
    check_neighbour_key();
    check_current_direct_map();
    if (failures) {
        std::printf("%d failures\n", failures);
        return 1;
    }
    std::printf("ok\n");
    return 0;
}
