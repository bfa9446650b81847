"""Schedule of the balanced scan (McNaughton's wrap-around rule over the tape
of n orbits x S steps), checked on the host through the library's own plan
and piece functions, the ones its kernel runs: every orbit's steps are
integrated exactly once and in order, each slot carries at most C steps, and
the two parts of every split orbit fall in different launches, the first part
earlier (this part needs no GPU)."""
import math

import numpy as np
import pytest

from paper_1802_00147_amd import pn

pytestmark = pytest.mark.skipif(not __import__("os").path.exists(pn.LIB_PATH), reason="library not built")


def slot_pieces(n, S, C, s):
    """Every piece of slot s, in slot-time order: (orbit, a, b, start)."""
    total = n * S
    length = min(C, total - s * C)
    tau, out = 0, []
    while tau < length:
        orbit, a, b, start = pn.balanced_piece(n, S, C, s, tau)
        assert start == tau and 0 <= a < b <= S and 0 <= orbit < n
        out.append((orbit, a, b, start))
        tau += b - a
    assert tau == length
    return out


def check_schedule(n, S, P):
    C, L = pn.balanced_plan(n, S, P)
    c = -(-C // L)
    assert C * P >= n * S and C > S and 2 <= L <= 16
    assert C - S >= c                                    # the condition that orders split parts
    if L > 2:                                            # the smallest launch count that satisfies it
        assert C - S < -(-C // (L - 1))
    used = -(-(n * S) // C)
    assert used <= P
    parts = {}
    for s in range(used):
        ps = slot_pieces(n, S, C, s)
        for k, (orbit, a, b, start) in enumerate(ps):
            parts.setdefault(orbit, []).append((a, b, s, start, k == 0, k == len(ps) - 1))
    assert sorted(parts) == list(range(n))
    for orbit, pl in parts.items():
        pl.sort()
        # The pieces of an orbit tile [0, S) exactly once.
        assert pl[0][0] == 0 and pl[-1][1] == S
        assert all(pl[i][1] == pl[i + 1][0] for i in range(len(pl) - 1))
        assert len(pl) <= 2
        if len(pl) == 2:
            (a0, b0, s0, t0, first0, _), (a1, b1, s1, t1, _, last1) = pl
            # First part at the start of slot s + 1, the rest at the end of
            # slot s: the record the first part saves (index s0) is the one the
            # second part loads (its slot + 1).
            assert s0 == s1 + 1 and first0 and t0 == 0 and last1 and t1 + (b1 - a1) == min(C, n * S - s1 * C)
            assert (t0 + (b0 - a0) - 1) // c < t1 // c  # written in an earlier launch than read
        else:
            assert pl[0][1] - pl[0][0] == S
    return C, L


@pytest.mark.parametrize("n,S,P", [(10, 7, 3), (98, 13, 16), (5, 100, 64), (1, 50, 1), (97, 1, 7),
                                   (1000, 3, 64), (64, 64, 64), (65, 64, 64), (33, 1000, 32), (7, 5, 2)])
def test_schedule_small(n, S, P):
    check_schedule(n, S, P)


def test_schedule_random():
    rng = np.random.default_rng(11)
    for _ in range(40):
        n = int(rng.integers(1, 300))
        S = int(rng.integers(1, 400))
        P = int(rng.integers(1, 200))
        check_schedule(n, S, P)


def test_plan_at_the_scan_sizes():
    """The 314 x 314 grids (98,596 orbits) on 65,536 and 32,768 slots: one
    wavefront per SIMD gives C = 3.009 S and two launches, two give 1.5045 S
    and three launches; the 4096 x 4096 grid divides evenly."""
    for S in (100_000, 1_000_000):
        C, L = pn.balanced_plan(98596, S, 32768)
        assert C == math.ceil(98596 * S / 32768) and L == 2
        C, L = pn.balanced_plan(98596, S, 65536)
        assert C == math.ceil(98596 * S / 65536) and L == 3
    C, L = pn.balanced_plan(4096 * 4096, 100_000, 32768)
    assert C == 512 * 100_000 and L == 2
    # Fewer orbits than slots: C is raised to S + ceil(S / 15), at most 16 launches.
    C, L = pn.balanced_plan(4096, 100_000, 65536)
    assert C == 100_000 + math.ceil(100_000 / 15) and L == 16


def test_plan_and_piece_errors():
    for args in ((0, 10, 4), (10, 0, 4), (10, 10, 0), (10, 10, (1 << 24) + 1), (1 << 35, 1 << 30, 4)):
        with pytest.raises(pn.PnError):
            pn.balanced_plan(*args)
    C, _ = pn.balanced_plan(10, 7, 3)
    for args in ((10, 7, C, 0, -1), (10, 7, C, 0, C), (10, 7, C, 3, 0), (10, 7, 7, 0, 0), (10, 7, C, -1, 0)):
        with pytest.raises(pn.PnError):
            pn.balanced_piece(*args)


def test_plan_at_the_overflow_guards():
    """Tapes up to 2^62 steps plan with both invariants; beyond the guards
    (n S or P C above 2^62) the plan is refused instead of wrapping."""
    for n, S, P in (((1 << 35), (1 << 26), 65536), (98596, 10 ** 12, 65536), (2, 3, 1 << 24)):
        C, L = pn.balanced_plan(n, S, P)
        assert C * P >= n * S and C - S >= -(-C // L) and 2 <= L <= 16
    for n, S, P in (((1 << 35), (1 << 27) + 1, 65536), (1, 1 << 40, 1 << 24)):
        with pytest.raises(pn.PnError):
            pn.balanced_plan(n, S, P)
