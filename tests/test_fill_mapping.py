"""Index arithmetic of the column-wise LDS table fill (host replay, no GPU).

Lane tid of a WG-lane workgroup keeps column c = tid mod tw of rows
r0 = tid / tw, r0 + R, ... (R = WG / tw rows per pass), its first row taken
as floor(tid * ceil(2^24 / tw) / 2^24) through a 32-bit high multiply of
tid << 8.  The replay checks that this quotient is exact for every lane id
and every table pitch a table can have, and that the lanes write every
entry e = r tw + c of a tw x rows table exactly once, from texel
(min(tx0 + c, W - 1), ty0 + r), with both halves of the two-entry trips."""
import numpy as np
import pytest


def _magic(tw: int) -> int:
    return (0x1000000 + tw - 1) // tw


def _first_row(tid: np.ndarray, tw: int) -> np.ndarray:
    # __umulhi((unsigned)tid << 8, m): the high 32 bits of a 64-bit product
    return (((tid.astype(np.uint64) << np.uint64(8)) * np.uint64(_magic(tw))) >> np.uint64(32)).astype(np.int64)


def test_magic_quotient_exact_for_every_lane_and_pitch():
    tid = np.arange(1024, dtype=np.int64)
    for tw in range(1, 2 * 9728 + 1):
        assert (_first_row(tid, tw) == tid // tw).all(), tw


def _replay(WG, W, tx0, ty0, tw, rows):
    R = WG // tw
    writes = {}
    for tid in range(WG):
        r0 = int(_first_row(np.array([tid]), tw)[0])
        if r0 >= R:
            continue
        c = tid - r0 * tw
        p = (ty0 + r0) * W + min(tx0 + c, W - 1)
        dp, de = R * W, R * tw
        e, r = tid, r0
        while r + R < rows:
            for pe, pp in ((e, p), (e + de, p + dp)):
                assert pe not in writes
                writes[pe] = pp
            p += 2 * dp
            e += 2 * de
            r += 2 * R
        if r < rows:
            assert e not in writes
            writes[e] = p
    return writes


@pytest.mark.parametrize("WG", [256, 512, 1024])
def test_every_entry_written_once_from_its_texel(WG):
    rng = np.random.default_rng(WG)
    cases = [(1, 1), (24, 1), (24, 200), (WG, 3), (WG - 8, 17), (40, 33), (72, 64)]
    cases += [(int(t), int(r)) for t, r in zip(rng.integers(1, WG + 1, 40), rng.integers(1, 120, 40))]
    for tw, rows in cases:
        W = int(rng.integers(tw // 2 + 1, 3 * tw + 2))
        tx0 = int(rng.integers(0, W))
        ty0 = int(rng.integers(0, 50))
        writes = _replay(WG, W, tx0, ty0, tw, rows)
        assert sorted(writes) == list(range(tw * rows)), (tw, rows)
        for e, p in writes.items():
            r, c = divmod(e, tw)
            assert p == (ty0 + r) * W + min(tx0 + c, W - 1), (tw, rows, e)
