"""A lane-level CPU model of the wave-run MTTKRP kernel's row walk (the row-advance
loop of mttkrp_wave_kernel), run on host data only.

A wave of 64 lanes is G groups of L lanes; step s gives group g the nonzero s*G + g
of the chunk's mode-sorted stream. The row being summed, `cur`, is wave-uniform;
each group keeps its share of it. When the last entry of a group of steps is still
in `cur`, the step is a plain accumulate; otherwise, per step, every row that ends
in it is closed: the shares are joined, the row is emitted, and the next row is read
from the lowest lane among the groups' first lanes whose row is past `cur` (a ballot,
then find-first-set, then readlane). On a sorted stream that lane always exists and
at most G rows end in one step; the kernel bounds the loop by both facts and, if
either fails, sets a device flag and leaves the loop. The model follows the same
lane arithmetic (ballot bits are lane numbers), so it checks that the walk emits
every row once on sorted streams and that an out-of-order stream ends the loop
with the flag set instead of spinning."""
import numpy as np
import pytest

WAVE = 64


def ballot(pred):
    """64-bit mask of the lanes whose predicate holds."""
    return sum(1 << lane for lane in range(WAVE) if pred[lane])


def ffs(mask):
    """1-based index of the lowest set bit (0 for an empty mask), as __ffsll."""
    return (mask & -mask).bit_length()


def walk(rows, vals, L, US, guard=True, spin_cap=10_000):
    """Sum vals per row over one chunk the way the kernel's row walk does.
    Returns (sums by row, flag, the most rows closed in one step)."""
    G = WAVE // L
    n = len(rows)
    lane = np.arange(WAVE)
    g_of, j_of = lane // L, lane % L
    tiles = -(-n // WAVE)
    last_row = rows[-1]
    out, flag, worst = {}, 0, 0
    cur = rows[0]
    acc = np.zeros(WAVE)  # every lane of a group holds the group's share

    def close(extra):
        total = sum(acc[g * L] + extra[g * L] for g in range(G))  # join the shares (group 0 stores)
        out[cur] = out.get(cur, 0.0) + total

    for t in range(tiles):
        base = t * WAVE
        # entries past the chunk carry its last row and add nothing
        er = np.array([rows[base + i] if base + i < n else last_row for i in range(WAVE)])
        ev = np.array([vals[base + i] if base + i < n else 0.0 for i in range(WAVE)])
        for m in range(L // US):
            mlast = er[(m + 1) * US * G - 1]  # readlane of the group of steps' last entry
            for u in range(US):
                src = (m * US + u) * G + g_of  # the entry each lane's group takes
                ru, vu = er[src], ev[src]
                if mlast == cur:
                    acc += vu
                    continue
                rl = er[(m * US + u) * G + G - 1]
                closed = 0
                while cur != rl:
                    close(np.where(ru == cur, vu, 0.0))
                    acc[:] = 0.0
                    ahead = ballot((j_of == 0) & (ru > cur))
                    closed += 1
                    if guard and (ahead == 0 or closed > G):
                        flag = 2
                        cur = rl
                        break
                    if not guard and closed > spin_cap:
                        raise RuntimeError("row walk did not end")
                    first_lane = ffs(ahead) - 1
                    cur = ru[first_lane] if first_lane >= 0 else cur
                worst = max(worst, closed)
                acc += np.where(ru == cur, vu, 0.0)
    close(np.zeros(WAVE))
    return out, flag, worst


def sorted_stream(rng, n, nrows, heavy=False):
    if heavy:  # a few long rows among many single nonzeros
        counts = rng.integers(1, 3, nrows)
        counts[rng.choice(nrows, 3, replace=False)] = rng.integers(100, 400, 3)
    else:
        counts = rng.integers(0, 6, nrows)
    rows = np.repeat(np.arange(nrows), counts)[:n]
    return rows, rng.integers(0, 8, rows.size).astype(np.float64)


@pytest.mark.parametrize("L,US", [(8, 8), (16, 2), (4, 4), (16, 4)])
@pytest.mark.parametrize("heavy", [False, True])
def test_walk_emits_each_row_once_on_sorted_streams(L, US, heavy):
    rng = np.random.default_rng(L * 10 + US + heavy)
    for _ in range(5):
        rows, vals = sorted_stream(rng, 2048, 900, heavy)
        out, flag, worst = walk(rows, vals, L, US)
        uniq = np.unique(rows)
        sums = np.bincount(rows, weights=vals)
        assert flag == 0
        assert sorted(out) == [int(r) for r in uniq]
        for r in uniq:
            assert out[int(r)] == sums[r]  # small integers: exact in any order
        assert worst <= WAVE // L


def test_many_rows_closing_in_one_step_stay_within_the_bound():
    """Every entry its own row: G rows end in each step, the most the bound allows."""
    for L in (1, 4, 8, 16):
        rows = np.arange(1024)
        out, flag, worst = walk(rows, np.ones(1024), L, min(L, 8))
        assert flag == 0 and worst == WAVE // L and len(out) == 1024


@pytest.mark.parametrize("L,US", [(8, 8), (16, 2)])
def test_out_of_order_stream_sets_the_flag_and_ends(L, US):
    """A stream whose rows go down inside a step leaves no group past `cur`: the ballot is
    empty. The bounded walk sets the flag and finishes the chunk; without the bound the
    walk would read lane -1 and never reach the step's last row."""
    G = WAVE // L
    rows = np.repeat(np.arange(0, 400, 2), 8)[:1024].copy()
    step = 37
    rows[step * G: step * G + G] = 10  # rows far below the current one ...
    rows[step * G + G - 1] = 5  # ... and a last entry below them
    vals = np.ones(rows.size)
    out, flag, _ = walk(rows, vals, L, US, guard=True)
    assert flag == 2
    with pytest.raises(RuntimeError):
        walk(rows, vals, L, US, guard=False, spin_cap=1000)
