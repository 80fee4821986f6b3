// Hilbert-curve order of the patch grid and cost-balanced curve segments.
//
// Section 3.1 and Fig. 2 of the paper: the patches lie along a Hilbert
// space-filling curve, each process owns one contiguous segment of it, and
// processes trade patches to even out their loads.  On one GPU the order is
// used for the work queue (patches of equal size are queued in curve order)
// and the segments are the partition a multi-GPU run would use.
//
// 2-D: a square of side 2^m is cut into quadrants traversed in the order
// lower-left (transposed sub-curve), upper-left, upper-right (sub-curve as
// is), lower-right (sub-curve reflected in the anti-diagonal), so the curve
// runs from cell (0, 0) to cell (side - 1, 0).  3-D: Skilling's transpose
// form of the Hilbert index (AIP Conf. Proc. 707, 2004), with the axes
// permuted so the curve runs from (0, 0, 0) to (side - 1, 0, 0).  Grids of
// 2^a x 2^b (x 2^c) patches are cut into squares (cubes) of the shortest side
// along the one longest axis, traversed in order; consecutive squares meet
// with a unit step.
#include "runtime.h"

#include <array>
#include <vector>

namespace pic {

namespace {

bool pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

// cell of position d of the curve over a side x side square
void square_cell(int side, int64_t d, int &x, int &y)
{
    if (side == 1) {
        x = y = 0;
        return;
    }
    const int h = side / 2;
    const int64_t q = (int64_t)h * h;
    const int digit = (int)(d / q);
    int a, b;
    square_cell(h, d % q, a, b);
    switch (digit) {
        case 0: x = b; y = a; break;                       // transposed
        case 1: x = a; y = b + h; break;
        case 2: x = a + h; y = b + h; break;
        default: x = 2 * h - 1 - b; y = h - 1 - a; break;  // anti-transposed
    }
}

// Skilling: Hilbert index in transpose form -> axis coordinates (in place)
void transpose_to_axes(std::array<uint32_t, 3> &X, int bits)
{
    const uint32_t N = 2u << (bits - 1);
    uint32_t t = X[2] >> 1;
    for (int i = 2; i > 0; --i) X[i] ^= X[i - 1];
    X[0] ^= t;
    for (uint32_t Q = 2; Q != N; Q <<= 1) {
        const uint32_t P = Q - 1;
        for (int i = 2; i >= 0; --i) {
            if (X[i] & Q) {
                X[0] ^= P;
            } else {
                t = (X[0] ^ X[i]) & P;
                X[0] ^= t;
                X[i] ^= t;
            }
        }
    }
}

std::array<uint32_t, 3> cube_raw(int side, int64_t d)
{
    int bits = 0;
    while ((1 << bits) < side) ++bits;
    std::array<uint32_t, 3> X{0, 0, 0};
    for (int b = 0; b < 3 * bits; ++b) {
        const uint32_t bit = (uint32_t)((d >> (3 * bits - 1 - b)) & 1);
        X[b % 3] |= bit << (bits - 1 - b / 3);
    }
    transpose_to_axes(X, bits);
    return X;
}

}  // namespace

int hilbert_patch_order(int nd, const int np[3], std::vector<int32_t> &out, std::string &why)
{
    const int64_t total = (int64_t)np[0] * np[1] * (nd == 3 ? np[2] : 1);
    out.assign(total, 0);
    for (int a = 0; a < nd; ++a)
        if (!pow2(np[a])) {
            why = "the Hilbert order needs power-of-two patch counts per axis";
            return PIC_ENOTSUP;
        }
    if (nd == 2) {
        const int side = std::min(np[0], np[1]);
        const bool along_x = np[0] >= np[1];
        const int64_t per = (int64_t)side * side;
        int64_t k = 0;
        for (int sq = 0; sq < std::max(np[0], np[1]) / side; ++sq)
            for (int64_t d = 0; d < per; ++d) {
                int a, b;
                square_cell(side, d, a, b);
                const int x = along_x ? sq * side + a : b, y = along_x ? b : sq * side + a;
                out[k++] = x + np[0] * y;
            }
        return PIC_OK;
    }
    int lng = 0;
    for (int a = 1; a < 3; ++a)
        if (np[a] > np[lng]) lng = a;
    const int o1 = (lng + 1) % 3, o2 = (lng + 2) % 3;
    const int side = std::min(np[o1], np[o2]);
    if (np[o1] != np[o2] || np[lng] < side) {
        why = "the 3-D Hilbert order needs two equal axes no longer than the third";
        return PIC_ENOTSUP;
    }
    const int lo1 = std::min(o1, o2), lo2 = std::max(o1, o2);  // the other axes in ascending order
    // frame: the raw curve ends one edge away from its start; that edge's
    // axis becomes the local first axis
    int perm[3] = {0, 1, 2};
    if (side > 1) {
        const std::array<uint32_t, 3> e = cube_raw(side, (int64_t)side * side * side - 1);
        int ax = 0;
        for (int a = 0; a < 3; ++a)
            if (e[a] != 0) ax = a;
        perm[0] = ax;
        int j = 1;
        for (int a = 0; a < 3; ++a)
            if (a != ax) perm[j++] = a;
    }
    const int64_t per = (int64_t)side * side * side;
    int64_t k = 0;
    for (int cb = 0; cb < np[lng] / side; ++cb)
        for (int64_t d = 0; d < per; ++d) {
            std::array<uint32_t, 3> r{0, 0, 0};
            if (side > 1) r = cube_raw(side, d);
            int c[3];
            c[lng] = cb * side + (int)r[perm[0]];
            c[lo1] = (int)r[perm[1]];
            c[lo2] = (int)r[perm[2]];
            out[k++] = c[0] + np[0] * (c[1] + np[1] * c[2]);
        }
    return PIC_OK;
}

void curve_segments(const int64_t *cost, int64_t n, int k, int64_t *bounds)
{
    __int128 total = 0;
    for (int64_t i = 0; i < n; ++i) total += cost[i];
    bounds[0] = 0;
    __int128 run = 0;
    int64_t i = 0;
    for (int j = 1; j < k; ++j) {
        // first position whose preceding costs reach j / k of the total
        while (i < n && run * k < total * j) run += cost[i++];
        bounds[j] = i;
    }
    bounds[k] = n;
}

}  // namespace pic
