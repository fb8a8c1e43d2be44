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

int main() {
    check_mix_lane();
    if (failures) {
        std::printf("%d failures\n", failures);
        return 1;
    }
    std::printf("ok\n");
    return 0;
}
