// psc_order.hip -- the order in which the (run, species, patch) units of the
// particle work are handed out: patches along a Hilbert-Peano space-filling
// curve (section "Dynamic load balancing using space filling curves"; the
// load-balancing figure with 16 x 16 patches).  Consecutive patches on the
// curve are neighbours in space, so a contiguous segment of the curve -- the
// eighth of the work items an XCD's queue owns, or the units of one
// persistent workgroup after the App. A split -- is a compact block of the
// domain rather than a strip.  Host code only.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <numeric>
#include <vector>

#include "psc_internal.h"

namespace psc {

// Index of the point x[0..n-1] (each coordinate below 2^bits) along the
// n-dimensional Hilbert curve, after Skilling's construction ("Programming
// the Hilbert curve", AIP Conf. Proc. 707, 2004).  The curve of a cube of
// side 2^bits is its eight (four in 2-d) half-size sub-cubes visited in Gray
// code order, each holding a reflected and axis-exchanged copy of the
// curve.  Going from the coarsest level to the finest, the reflection or
// exchange a point's sub-cube applies is undone on the finer bits of the
// coordinates; the coordinates then hold the Gray code of the index one
// bit-plane per level, which is decoded and read out level by level with
// coordinate 0 as the most significant bit of each digit.
static uint64_t hilbert_index(int n, int bits, uint32_t x[3]) {
    if (bits <= 0) return 0;
    const uint32_t top = 1u << (bits - 1);
    for (uint32_t q = top; q > 1; q >>= 1) {
        const uint32_t finer = q - 1;
        for (int i = 0; i < n; ++i) {
            if (x[i] & q) {
                x[0] ^= finer;                              // reflection
            } else {
                const uint32_t t = (x[0] ^ x[i]) & finer;   // exchange of axes 0 and i
                x[0] ^= t;
                x[i] ^= t;
            }
        }
    }
    // Gray decode across the coordinates, then across the levels
    for (int i = 1; i < n; ++i) x[i] ^= x[i - 1];
    uint32_t flip = 0;
    for (uint32_t q = top; q > 1; q >>= 1)
        if (x[n - 1] & q) flip ^= q - 1;
    for (int i = 0; i < n; ++i) x[i] ^= flip;
    uint64_t h = 0;
    for (int b = bits - 1; b >= 0; --b)
        for (int i = 0; i < n; ++i) h = (h << 1) | ((x[i] >> b) & 1u);
    return h;
}

// Patches of a grid of np[0] x np[1] x np[2] (x fastest, np[0] == 1 for a
// 2-d run) in Hilbert order: the curve of the smallest power-of-two cube
// that holds the grid, restricted to the grid.  The grid's axes are mapped
// onto the curve's coordinates by whichever permutation leaves the fewest
// consecutive pairs that are not face neighbours: none for a cube of side
// 2^k, and none for boxes that fill a leading part of the curve (2:1 in 2-d;
// 2:1:1 and 2:2:1 in 3-d, e.g. 32 x 16 patches); a few jumps otherwise.
void hilbert_patch_order(int dim, const int np[3], std::vector<int32_t> &order) {
    const int n_patch = np[0] * np[1] * np[2];
    order.resize(n_patch);
    std::iota(order.begin(), order.end(), 0);
    if (n_patch <= 1) return;
    int axes[3] = {0, 1, 2};
    const int na = dim == 3 ? 3 : 2;
    const int *act = dim == 3 ? axes : axes + 1;    // active grid axes
    int side = 1, bits = 0;
    for (int k = 0; k < 3; ++k)
        while (side < np[k]) side <<= 1, ++bits;
    int perm[3] = {0, 1, 2};
    std::vector<uint64_t> key(n_patch);
    std::vector<int32_t> best, cand(n_patch);
    int64_t best_jumps = -1;
    do {
        for (int p = 0; p < n_patch; ++p) {
            const int c[3] = {p % np[0], (p / np[0]) % np[1], p / (np[0] * np[1])};
            uint32_t x[3] = {0, 0, 0};
            for (int i = 0; i < na; ++i) x[i] = (uint32_t)c[act[perm[i]]];
            key[p] = hilbert_index(na, bits, x);
        }
        std::iota(cand.begin(), cand.end(), 0);
        std::sort(cand.begin(), cand.end(), [&](int32_t a, int32_t b) { return key[a] < key[b]; });
        int64_t jumps = 0;
        for (int t = 1; t < n_patch; ++t) {
            const int a = cand[t - 1], b = cand[t];
            const int d = std::abs(a % np[0] - b % np[0]) + std::abs((a / np[0]) % np[1] - (b / np[0]) % np[1]) +
                          std::abs(a / (np[0] * np[1]) - b / (np[0] * np[1]));
            jumps += d != 1;
        }
        if (best_jumps < 0 || jumps < best_jumps) {
            best_jumps = jumps;
            best = cand;
        }
    } while (std::next_permutation(perm, perm + na));
    order = best;
}

}  // namespace psc

extern "C" psc_status psc_hilbert_order(int dim, const int32_t np[3], int32_t *order) {
    if ((dim != 2 && dim != 3) || !np || !order) return PSC_ERR_INVALID;
    if (np[0] < 1 || np[1] < 1 || np[2] < 1 || (dim == 2 && np[0] != 1)) return PSC_ERR_INVALID;
    if ((int64_t)np[0] * np[1] * np[2] > (int64_t(1) << 24)) return PSC_ERR_INVALID;
    const int n[3] = {np[0], np[1], np[2]};
    std::vector<int32_t> o;
    psc::hilbert_patch_order(dim, n, o);
    std::copy(o.begin(), o.end(), order);
    return PSC_OK;
}
