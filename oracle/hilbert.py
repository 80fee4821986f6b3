"""Oracle: Hilbert-curve order of the patches and cost-balanced segments of it
(test infrastructure only; the product library never loads it).

The paper (section 3.1 and Fig. 2) arranges the patches along a Hilbert
space-filling curve; each process owns one contiguous segment of the curve,
and processes trade patches to even out their loads.  For a 32 x 32 patch
grid the curve visits every patch once, starting at patch (0, 0) and ending
at patch (31, 0).  The paper does not give the curve for non-square grids or
the load measure; the readings used here:

* 2-D grid of 2^a x 2^b patches: the longer axis is cut into squares of the
  shorter side, each traversed by the square curve from its corner (0, 0) to
  (side - 1, 0) of its own frame, squares in order along the longer axis;
  consecutive squares meet with a unit step.
* 3-D grid of 2^a x 2^b x 2^c patches with one axis longest: cubes of the
  common side along that axis, each traversed by the 3-D curve of Skilling
  (AIP Conf. Proc. 707, 2004: the "transpose" form of the Hilbert index)
  oriented from its corner (0, 0, 0) to (side - 1, 0, 0).
* Segments: k contiguous pieces of the curve; piece j starts at the first
  curve position whose preceding costs reach j / k of the total, so every
  piece costs at most total / k plus the largest single patch cost.

Pins (tests/test_oracle_hilbert.py): the Fig. 2 end points and that every
patch is visited once with unit steps, for square, rectangular and 3-D grids;
the segment bound above and brute-force optimality bounds on small inputs.
Plain Python loops: the grids involved have at most a few ten thousand
patches.
"""
from __future__ import annotations


def _is_pow2(v: int) -> bool:
    return v > 0 and (v & (v - 1)) == 0


def square_point(side: int, d: int):
    """Cell (x, y) at position d of the Hilbert curve over a side x side grid
    (side a power of two).  The curve is built bottom-up: at each scale s the
    quadrant is read from two bits of d, the partial point is reflected and
    transposed into that quadrant's frame, then offset by the quadrant."""
    x = y = 0
    t = d
    s = 1
    while s < side:
        qx = 1 & (t // 2)
        qy = 1 & (t ^ qx)
        if qy == 0:
            if qx == 1:
                x = s - 1 - x
                y = s - 1 - y
            x, y = y, x
        x += s * qx
        y += s * qy
        t //= 4
        s *= 2
    return x, y


def _transpose_to_axes(X, bits):
    """Skilling's inverse transform: Hilbert index in transpose form (one word
    per axis, index bits distributed across the axes from the top) to axis
    coordinates, in place."""
    n = len(X)
    N = 2 << (bits - 1)
    # Gray decode by H ^ (H / 2)
    t = X[n - 1] >> 1
    for i in range(n - 1, 0, -1):
        X[i] ^= X[i - 1]
    X[0] ^= t
    # undo excess work
    Q = 2
    while Q != N:
        P = Q - 1
        for i in range(n - 1, -1, -1):
            if X[i] & Q:
                X[0] ^= P
            else:
                t = (X[0] ^ X[i]) & P
                X[0] ^= t
                X[i] ^= t
        Q <<= 1
    return X


def cube_point_raw(side: int, d: int):
    """Axis coordinates of position d of Skilling's 3-D Hilbert curve over a
    side^3 grid (side a power of two, side >= 2)."""
    bits = side.bit_length() - 1
    # index bits, most significant first, go round-robin to axes 0, 1, 2
    X = [0, 0, 0]
    for b in range(3 * bits):
        bit = (d >> (3 * bits - 1 - b)) & 1
        axis = b % 3
        X[axis] |= bit << (bits - 1 - b // 3)
    return tuple(_transpose_to_axes(X, bits))


def _cube_frame(side: int):
    """An axis permutation and reflections that take the raw 3-D curve to one
    running from (0, 0, 0) to (side - 1, 0, 0): the raw curve starts at the
    origin and ends at a corner one unit edge away."""
    s0 = cube_point_raw(side, 0)
    s1 = cube_point_raw(side, side ** 3 - 1)
    assert s0 == (0, 0, 0)
    axis = [a for a in range(3) if s1[a] != 0]
    assert len(axis) == 1 and s1[axis[0]] == side - 1
    a = axis[0]
    perm = [a] + [b for b in range(3) if b != a]   # new axis k reads raw axis perm[k]
    return perm


def cube_point(side: int, d: int):
    perm = _cube_frame(side)
    p = cube_point_raw(side, d)
    return tuple(p[perm[k]] for k in range(3))


def patch_order(np_):
    """Patch ids (x + nx (y + ny z)) in curve order for a grid of np_ patches
    (2 or 3 entries, powers of two; in 3-D one axis at least as long as the
    two others, which must be equal)."""
    nd = len(np_)
    if not all(_is_pow2(v) for v in np_):
        raise ValueError("patch counts must be powers of two")
    if nd == 2:
        nx, ny = np_
        side = min(nx, ny)
        long_x = nx >= ny
        out = []
        for sq in range(max(nx, ny) // side):
            for d in range(side * side):
                a, b = square_point(side, d)
                if long_x:
                    x, y = sq * side + a, b
                else:
                    # transposed frame: the curve runs along y
                    x, y = b, sq * side + a
                out.append(x + nx * y)
        return out
    nx, ny, nz = np_
    side = min(np_)
    longest = max(range(3), key=lambda a: np_[a])
    others = [a for a in range(3) if a != longest]
    if np_[others[0]] != side or np_[others[1]] != side:
        raise ValueError("3-D grids need two equal axes no longer than the third")
    out = []
    for cb in range(np_[longest] // side):
        for d in range(side ** 3):
            p = cube_point(side, d) if side > 1 else (0, 0, 0)
            c = [0, 0, 0]
            c[longest] = cb * side + p[0]
            c[others[0]] = p[1]
            c[others[1]] = p[2]
            out.append(c[0] + nx * (c[1] + ny * c[2]))
    return out


def segments(costs, k):
    """Boundaries b_0 = 0 <= b_1 <= ... <= b_k = n of k contiguous pieces of a
    sequence of non-negative costs: b_j is the first position i whose
    preceding costs sum to at least j / k of the total."""
    n = len(costs)
    total = sum(costs)
    bounds = [0]
    run = 0
    i = 0
    for j in range(1, k):
        # smallest i with sum(costs[:i]) * k >= j * total (exact integer test)
        while i < n and run * k < j * total:
            run += costs[i]
            i += 1
        bounds.append(i)
    bounds.append(n)
    return bounds
