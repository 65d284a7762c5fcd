"""Host logic of the specialised kernels' gather schedules (no GPU needed).

bcs_schedule_describe returns the schedule the library builds for a
pattern; these tests check it independently: every stored entry of the solved
matrix (A, or A^T for the adjoint) is gathered exactly once, at a step owned
by its own row's lane and slot (or the two slots of a spanning row), with its
own column, the diagonal left out exactly when the diagonal shape is used, and
the plain sliced-ELL deal has the slot lengths its definition gives.
"""
import numpy as np
import pytest

from workload import gen_mechanism

bcs = pytest.importorskip("paper_2405_17363_amd")

SHAPES = [0, 1, 2, 3]


def entries(rp, ci, transpose):
    """{CSR position: (row, column)} of the solved matrix."""
    out = {}
    for i in range(len(rp) - 1):
        for k in range(rp[i], rp[i + 1]):
            out[k] = (int(ci[k]), i) if transpose else (i, int(ci[k]))
    return out


def row_lengths(rp, ci, transpose):
    n = len(rp) - 1
    if not transpose:
        return np.diff(rp)
    return np.bincount(ci, minlength=n)


@pytest.mark.parametrize("n,R", [(30, 50), (80, 150), (200, 400)])
@pytest.mark.parametrize("lanes", [16, 32, 64])
@pytest.mark.parametrize("transpose", [False, True])
@pytest.mark.parametrize("shapes", SHAPES)
def test_every_entry_gathered_once_by_its_row(n, R, lanes, transpose, shapes):
    m = gen_mechanism(n, R)
    d = bcs.schedule_describe(m.row_ptr, m.col_idx, lanes, transpose, shapes)
    rpl, seg, row, pos, col = d["rows_per_lane"], d["seg"], d["row"], d["pos"], d["col"]
    assert rpl == -(-n // lanes)
    assert d["steps"] == seg.sum() and seg.min() >= 1
    assert d["shape"] & ~shapes == 0
    starts = np.concatenate([[0], np.cumsum(seg)])
    owner = np.full((d["steps"], lanes), -1)
    for j in range(rpl):
        for lane in range(lanes):
            r = row[j, lane]
            if r == -2:
                assert j == 1 and row[0, lane] >= 0 and d["shape"] & bcs.BCS_SCHED_SPAN
                owner[starts[1]:starts[2], lane] = row[0, lane]
            elif r >= 0:
                owner[starts[j]:starts[j + 1], lane] = r
            else:
                assert r == -1
    assert sorted(row[row >= 0].tolist()) == list(range(n))
    split = bool(d["shape"] & bcs.BCS_SCHED_DIAG)
    seen = {}
    for s in range(d["steps"]):
        for lane in range(lanes):
            p = int(pos[s, lane])
            if p < 0:
                continue
            assert p not in seen, (s, lane, p)
            seen[p] = (int(owner[s, lane]), int(col[s, lane]))
    expect = {k: rc for k, rc in entries(m.row_ptr, m.col_idx, transpose).items() if not (split and rc[0] == rc[1])}
    assert seen == expect


@pytest.mark.parametrize("transpose", [False, True])
@pytest.mark.parametrize("lanes", [16, 32, 64])
def test_plain_deal_slot_lengths_and_shapes_never_longer(lanes, transpose):
    m = gen_mechanism(80, 150)
    lens = np.sort(row_lengths(m.row_ptr, m.col_idx, transpose))[::-1]
    rpl = -(-80 // lanes)
    for shapes, minus in ((0, 0), (bcs.BCS_SCHED_DIAG, 1)):
        want = [max(1, int(lens[j * lanes:(j + 1) * lanes].max()) - minus) for j in range(rpl)]
        d = bcs.schedule_describe(m.row_ptr, m.col_idx, lanes, transpose, shapes)
        assert d["seg"].tolist() == want and d["shape"] == shapes
    plain = bcs.schedule_describe(m.row_ptr, m.col_idx, lanes, transpose, 0)["steps"]
    for shapes in SHAPES:
        assert bcs.schedule_describe(m.row_ptr, m.col_idx, lanes, transpose, shapes)["steps"] <= plain


def test_n80_at_32_lanes_spans_and_drops_the_diagonal():
    m = gen_mechanism(80, 150)
    plain = bcs.schedule_describe(m.row_ptr, m.col_idx, 32, False, 0)
    shaped = bcs.schedule_describe(m.row_ptr, m.col_idx, 32, False, bcs.BCS_SCHED_SPAN | bcs.BCS_SCHED_DIAG)
    assert plain["steps"] == 33 and shaped["steps"] == 26
    assert shaped["shape"] == bcs.BCS_SCHED_SPAN | bcs.BCS_SCHED_DIAG
    assert np.count_nonzero(shaped["row"][1] == -2) > 0


def test_diagonal_kept_when_a_row_lacks_it():
    rp = np.array([0, 2, 3, 5], np.int32)   # row 1 has no diagonal
    ci = np.array([0, 2, 0, 1, 2], np.int32)
    d = bcs.schedule_describe(rp, ci, 16, False, bcs.BCS_SCHED_DIAG)
    assert d["shape"] == 0 and sorted(d["pos"][d["pos"] >= 0].tolist()) == list(range(5))


@pytest.mark.parametrize("lanes,transpose,shapes", [(8, 0, 0), (32, 4, 0), (32, 0, 4)])
def test_bad_arguments_rejected(lanes, transpose, shapes):
    m = gen_mechanism(30, 50)
    with pytest.raises(bcs.BcsError):
        bcs.schedule_describe(m.row_ptr, m.col_idx, lanes, transpose, shapes)
