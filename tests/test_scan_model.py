"""The y/z distance pass's algorithm, modelled step for step in Python and
checked against the definition (host only; no GPU, no oracle).

The pass computes g(i) = min_j max(|i-j|, f(j)) over one line (the max-min
recurrence of the separable chessboard distance transform, Sec. 3.1).  The
kernels run it as a forward one-sided pass F(i) = min_{j<=i} max(i-j, f(j))
followed by the same pass backwards over F, each in one sweep that keeps
v = F(i-1), a witness W and a table last[w] of the latest position holding
value w.  On an advance the witness becomes the table entry last[v+1] alone,
with no max against the old witness; with that rule the witness after every
step equals last[F(i)] read after the step's own write, so each step writes
last[f(i)] = i, sets F(i) = min(f(i), min(v+1, max(v, i-W))) and reads
W = last[F(i)].  The split variant runs the forward and backward passes at once on two lanes, each
first over its half of the line and then over the half the other has done,
with values clamped at min(m, 255) and the line's minimum as the result
wherever every value is at least that clamp; the one-lane register kernel
clamps the same way, so its table needs only min(m, 255) + 1 rows.  These
models mirror that logic
so a change to it can be checked here first."""
import numpy as np
import pytest


def brute(f):
    f = np.asarray(f, dtype=np.int64)
    i = np.arange(len(f))
    return np.minimum(np.maximum(np.abs(i[:, None] - i[None, :]), f[None, :]).min(axis=1), 255)


class Lane:
    """One lane's scan state: v = F(i-1) and its witness W = last[v]."""

    def __init__(self, rows, v0):
        self.tbl = [0] * rows
        self.v, self.W = v0, 0

    def step(self, i, fi):
        self.tbl[fi] = i
        v = self.v
        X = min(v + 1, max(v, i - self.W))
        self.v = min(fi, X)
        self.W = self.tbl[self.v]
        return self.v


class SelectLane:
    """The same pass with the witness chosen among its candidates: position
    i on a new minimum, last[v+1] (read before the step's write) on an
    advance, else the old witness."""

    def __init__(self, rows, v0):
        self.tbl = [0] * rows
        self.v, self.W = v0, 0

    def step(self, i, fi):
        v = self.v
        adv = (i - self.W) > v
        X = v + (1 if adv else 0)
        cand = self.tbl[v + 1] if v + 1 < len(self.tbl) else 0
        self.tbl[fi] = i
        self.W = i if fi <= X else (cand if adv else self.W)
        self.v = min(fi, X)
        return self.v


def one_sided(col, rows=256):
    lane = Lane(rows, col[0])
    out = [col[0]]
    for i in range(1, len(col)):
        out.append(lane.step(i, col[i]))
    return out


def two_sided(f):
    fwd = one_sided([int(x) for x in f])
    return np.array(one_sided(fwd[::-1])[::-1])


def split(f):
    m = len(f)
    vmax, h = min(m, 255), m // 2
    tile = [int(x) for x in f]
    F, B = Lane(vmax + 3, min(tile[0], vmax)), Lane(vmax + 3, min(tile[m - 1], vmax))
    raw = [tile[0], tile[m - 1]]

    def run(lane, pos, i, k):
        r = tile[pos]
        tile[pos] = lane.step(i, min(r, vmax))
        if k is not None:
            raw[k] = min(raw[k], r)

    for i in range(1, h):                      # phase 1: each lane over its half
        run(F, i, i, 0)
        run(B, m - 1 - i, i, 1)
    if m - h > h:
        run(B, m - 1 - h, h, 1)
    lmin = min(raw)
    if m - h > h:
        run(F, h, h, None)
    for i in range(m - h, m):                  # phase 2: over the half the other lane did
        run(F, i, i, None)
        run(B, m - 1 - i, i, None)
    if lmin >= vmax:                           # every value >= the clamp: the line's minimum
        tile = [lmin] * m
    return np.array(tile)


def lines(seed, count, max_m=256):
    rng = np.random.default_rng(seed)
    for k in range(count):
        m = int(rng.integers(1, max_m + 1))
        kind = k % 6
        if kind == 0:
            f = rng.integers(0, 256, m)
        elif kind == 1:                       # x distances: sparse zeros, the rest capped
            f = np.where(rng.random(m) < 0.05, 0, 255)
        elif kind == 2:
            f = np.minimum(255, rng.integers(0, 40, m) + rng.integers(0, 3) * 100)
        elif kind == 3:                       # a distance ramp with noise
            f = np.minimum(255, np.abs(np.arange(m) - rng.integers(0, m)) + rng.integers(0, 5, m))
        elif kind == 4:                       # every value >= m (the split pass's fix-up)
            f = rng.integers(m, 256, m) if m < 256 else np.full(m, 255)
        else:                                 # values around m
            f = np.minimum(255, rng.integers(max(0, m - 3), m + 3, m))
        yield f


@pytest.mark.parametrize("seed", [1, 2])
def test_two_sided_scan_matches_definition(seed):
    for f in lines(seed, 300):
        np.testing.assert_array_equal(two_sided(f), brute(f), err_msg=str(list(f)))


@pytest.mark.parametrize("seed", [3, 4])
def test_split_scan_matches_definition(seed):
    for f in lines(seed, 300):
        np.testing.assert_array_equal(split(f), brute(f), err_msg=str(list(f)))


def test_witness_is_the_table_entry_of_the_value():
    # the step that reads W = last[F(i)] keeps the same witness as the rule
    # that picks among i, last[v+1] and the old witness, at every step
    for seed in (5, 6):
        for f in lines(seed, 200):
            a, b = Lane(257, 511), SelectLane(257, 511)
            for i, fi in enumerate(int(x) for x in f):
                assert a.step(i, fi) == b.step(i, fi)
                assert a.W == b.W, (list(f), i)


def test_scan_edge_lines():
    for f in ([0], [255], [7], [0, 255], [255, 0], [3, 3], [255] * 256, [0] * 256,
              [255] * 255 + [0], [0] + [255] * 255, list(range(256)), list(range(255, -1, -1))):
        np.testing.assert_array_equal(two_sided(f), brute(f))
        np.testing.assert_array_equal(split(f), brute(f))


def test_longer_lines_with_wide_table():
    # lines over 256 positions keep positions beyond 255 (16-bit table entries)
    rng = np.random.default_rng(9)
    for m in (257, 300):
        f = np.where(rng.random(m) < 0.02, 0, 255)
        np.testing.assert_array_equal(two_sided(f), brute(f))


def _padded_words(f, nch):
    """A line as the register kernels hold it: 4*nch words of 4 bytes, the
    positions past the line repeating its last value."""
    last = len(f) - 1
    return [[int(f[min(4 * r + k, last)]) for k in range(4)] for r in range(4 * nch)]


def registers_one_lane(f):
    """The one-lane register kernel: the line padded to whole chunks of 16,
    a forward pass from a start state above every value over the values
    clamped at s = min(m, 255) (a table of s + 1 rows; the line's minimum
    kept on the side), then a backward pass from the padded end (positions
    counted from it) whose stores take max(result, fix), fix being the
    line's minimum when every value is at least s and 0 otherwise; stores of
    padded positions go to the last position before its own store."""
    m = len(f)
    nch = -(-m // 16)
    pend = 16 * nch - 1
    s = min(m, 255)
    w = _padded_words(f, nch)
    fwd = Lane(s + 1, 511)
    lmin = 255
    for p in range(pend + 1):
        raw = w[p // 4][p % 4]
        lmin = min(lmin, raw)
        w[p // 4][p % 4] = fwd.step(p, min(raw, s))
    fix = lmin if lmin >= s else 0
    bwd = Lane(s + 1, 511)
    out = [None] * m
    for p in range(pend, -1, -1):
        out[min(p, m - 1)] = max(bwd.step(pend - p, w[p // 4][p % 4]), fix)
    return np.array(out)


def registers_pairs(f):
    """The two-lane register kernel: both lanes load the padded line, the
    upper lane reverses it (register r, byte k = position pend - 4r - k);
    phase 1 runs steps 0 .. H-1 (registers 0 .. 2*nch-1) on each lane's own
    data; the lanes swap halves (register r >= 2*nch takes the other lane's
    register 4*nch-1-r, byte-reversed); phase 2 runs steps H .. 2H-1; the
    upper lane's results are brought back into order and stored at positions
    0 .. H-1, the lower lane's at H .. pend, last first."""
    m = len(f)
    nch = -(-m // 16)
    NW, H = 4 * nch, 8 * nch
    assert nch >= 2
    lo, up = _padded_words(f, nch), _padded_words(f, nch)
    for j in range(NW // 2):
        a, b = up[j], up[NW - 1 - j]
        up[j], up[NW - 1 - j] = b[::-1], a[::-1]
    L, U = Lane(256, 511), Lane(256, 511)

    def phase(r0, r1):
        for r in range(r0, r1):
            for k in range(4):
                s = 4 * r + k
                lo[r][k] = L.step(s, lo[r][k])
                up[r][k] = U.step(s, up[r][k])

    phase(0, NW // 2)
    assert 4 * (NW // 2) == H
    for r in range(NW // 2, NW):
        lo[r], up[r] = up[NW - 1 - r][::-1], lo[NW - 1 - r][::-1]
    phase(NW // 2, NW)
    for j in range(NW // 2):
        up[j] = up[NW - 1 - j][::-1]
    out = [None] * m
    for r in range(NW // 2):
        for k in range(4):
            assert 4 * r + k < m
            out[4 * r + k] = up[r][k]
    for r in range(NW - 1, NW // 2 - 1, -1):
        for k in range(3, -1, -1):
            out[min(4 * r + k, m - 1)] = lo[r][k]
    return np.array(out)


def registers_pairs_slots(f):
    """The two-lane register kernel on rows that are staged through LDS: the
    tile's positions go to slots of one position each, slot s < H holding
    position s and slot H + s position pend - s (positions past the line
    repeat its last value); the lower lane reads slots 0 .. H-1 and the upper
    lane slots H .. 2H-1, each already in its own step order; phases and swap
    as in registers_pairs; step H + s of the lower lane goes back to slot s
    (position H + s) and of the upper lane to slot H + s (position H-1-s),
    from where the positions below m are stored."""
    m = len(f)
    nch = -(-m // 16)
    NW, H = 4 * nch, 8 * nch
    assert nch >= 2 and H <= m
    ks = (16 * nch + 31) // 32
    slots = [None] * (2 * H)
    for r in range(32 * ks):
        if r < 2 * H:
            slots[r if r < H else 3 * H - 1 - r] = int(f[min(r, m - 1)])
    lo = [[slots[4 * j + k] for k in range(4)] for j in range(NW // 2)] + [None] * (NW // 2)
    up = [[slots[H + 4 * j + k] for k in range(4)] for j in range(NW // 2)] + [None] * (NW // 2)
    L, U = Lane(256, 511), Lane(256, 511)

    def phase(r0, r1):
        for r in range(r0, r1):
            for k in range(4):
                s = 4 * r + k
                lo[r][k] = L.step(s, lo[r][k])
                up[r][k] = U.step(s, up[r][k])

    phase(0, NW // 2)
    for r in range(NW // 2, NW):
        lo[r], up[r] = up[NW - 1 - r][::-1], lo[NW - 1 - r][::-1]
    phase(NW // 2, NW)
    back = [None] * (2 * H)
    for r in range(NW // 2, NW):
        for k in range(4):
            back[4 * (r - NW // 2) + k] = lo[r][k]
            back[H + 4 * (r - NW // 2) + k] = up[r][k]
    return np.array([back[r - H] if r >= H else back[2 * H - 1 - r] for r in range(m)])


@pytest.mark.parametrize("seed", [5, 6])
def test_register_kernels_match_definition(seed):
    for f in lines(seed, 300):
        np.testing.assert_array_equal(registers_one_lane(f), brute(f), err_msg=str(list(f)))
        if len(f) > 16:
            np.testing.assert_array_equal(registers_pairs(f), brute(f), err_msg=str(list(f)))
            np.testing.assert_array_equal(registers_pairs_slots(f), brute(f), err_msg=str(list(f)))


def test_register_kernels_every_chunk_count():
    # every line length 17..256 (odd and even chunk counts, the split point
    # at 8*nch), sparse and dense lines
    rng = np.random.default_rng(21)
    for m in range(2, 257):
        for f in (np.where(rng.random(m) < 0.04, 0, 255), rng.integers(0, 256, m)):
            np.testing.assert_array_equal(registers_one_lane(f), brute(f), err_msg=f"m={m}")
            if m > 16:
                np.testing.assert_array_equal(registers_pairs(f), brute(f), err_msg=f"m={m}")
                np.testing.assert_array_equal(registers_pairs_slots(f), brute(f), err_msg=f"m={m}")
