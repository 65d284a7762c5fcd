"""Host logic of the ILU(0) kernel (no GPU needed).

The kernel factorises each cell by a program that the library builds once per
pattern (bcs_ilu_describe) and applies the factors through gather schedules
of the strict triangles (bcs_schedule_describe with BCS_PART_LOWER / UPPER).
These tests check both independently of the library:

* the program, interpreted here step by step in plain float64, turns A into
  exactly the oracle's ILU(0) factors (the same operations in the same order,
  so bitwise);
* its steps are well formed: one operation per changed entry, no operation
  reads a value written in its own step, the divisor is the column's pivot
  below the diagonal and the constant 1 above it;
* every strict-triangle entry is gathered exactly once, by a lane and slot
  that own its row, with its own column.
"""
import numpy as np
import pytest

import oracle
from workload import gen_mechanism

bcs = pytest.importorskip("paper_2405_17363_amd")


def unpack(words, widths, lanes):
    """[(heads[lanes], terms[w][lanes])] per step, as (lo, hi) 16-bit pairs."""
    steps, o = [], 0
    for w in widths:
        head = words[o:o + lanes]
        o += lanes
        terms = [words[o + q * lanes:o + (q + 1) * lanes] for q in range(w)]
        o += w * lanes
        steps.append((head, terms))
    assert o == len(words)
    return steps


def run_program(steps, A, nnz):
    """Apply the program to A (CSR values) in plain float64."""
    F = np.concatenate([np.asarray(A, np.float64), [0.0, 1.0, 0.0]])
    for head, terms in steps:
        new = {}
        for lane in range(len(head)):
            t, d = int(head[lane] & 0xFFFF), int(head[lane] >> 16)
            acc = F[t]
            for tw in terms:
                acc = acc - F[int(tw[lane] & 0xFFFF)] * F[int(tw[lane] >> 16)]
            new[t] = acc / F[d]  # steps read only values final before them
        for t, v in new.items():
            F[t] = v
    return F[:nnz]


def cell_matrix(m, seed):
    rng = np.random.default_rng(seed)
    J = rng.standard_normal(len(m.col_idx)) * 10.0 ** rng.uniform(-3, 1, len(m.col_idx))
    return oracle.form_a(m.row_ptr, m.col_idx, J, rng.uniform(0.1, 2.0))


@pytest.mark.parametrize("n,R", [(30, 50), (80, 150), (200, 400)])
@pytest.mark.parametrize("lanes", [16, 32, 64])
def test_program_reproduces_the_oracle_factors_bitwise(n, R, lanes):
    m = gen_mechanism(n, R)
    P = bcs.ilu_describe(m.row_ptr, m.col_idx, lanes)
    steps = unpack(P["words"], P["widths"], lanes)
    for seed in range(3):
        A = cell_matrix(m, seed)
        got = run_program(steps, A, len(m.col_idx))
        want = oracle.ilu0(m.row_ptr, m.col_idx, A)
        assert np.array_equal(got, want), np.max(np.abs(got - want))


@pytest.mark.parametrize("n,R", [(30, 50), (80, 150)])
@pytest.mark.parametrize("lanes", [16, 32, 64])
def test_program_steps_are_well_formed(n, R, lanes):
    m = gen_mechanism(n, R)
    rp, ci = m.row_ptr, m.col_idx
    nnz = len(ci)
    zero, unit, junk = nnz, nnz + 1, nnz + 2
    rows = np.repeat(np.arange(n), np.diff(rp))
    diag = {i: k for k in range(nnz) for i in [rows[k]] if ci[k] == i}
    P = bcs.ilu_describe(rp, ci, lanes)
    steps = unpack(P["words"], P["widths"], lanes)
    targets = []
    for head, terms in steps:
        mine = set()
        for lane in range(lanes):
            t, d = int(head[lane] & 0xFFFF), int(head[lane] >> 16)
            if t == junk:
                assert d == unit and all(int(tw[lane]) == zero | zero << 16 for tw in terms)
                continue
            i, j = rows[t], ci[t]
            assert d == (diag[j] if i > j else unit)
            mine.add(t)
            targets.append(t)
        for lane in range(lanes):
            reads = [int(head[lane] >> 16)] + [int(tw[lane]) & 0xFFFF for tw in terms] + \
                    [int(tw[lane]) >> 16 for tw in terms]
            assert not (set(reads) & mine), "an operation reads a value written in its own step"
    # one operation per entry the elimination changes: every strict-lower
    # entry, and the upper entries with at least one term
    changed = set()
    at = {(rows[k], ci[k]): k for k in range(nnz)}
    for k in range(nnz):
        i, j = rows[k], ci[k]
        if i > j or any((i, q) in at and (q, j) in at for q in range(min(i, j))):
            changed.add(k)
    assert sorted(targets) == sorted(changed)


def test_dense_pattern_program_is_lu_without_pivoting():
    n = 6
    rp = np.arange(0, n * n + 1, n, dtype=np.int32)
    ci = np.tile(np.arange(n, dtype=np.int32), n)
    rng = np.random.default_rng(3)
    A = rng.standard_normal((n, n)) + n * np.eye(n)
    P = bcs.ilu_describe(rp, ci, 16)
    F = run_program(unpack(P["words"], P["widths"], 16), A.ravel(), n * n).reshape(n, n)
    L = np.tril(F, -1) + np.eye(n)
    U = np.triu(F)
    assert np.allclose(L @ U, A, rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("n,R", [(30, 50), (80, 150), (200, 400)])
@pytest.mark.parametrize("lanes", [16, 32, 64])
@pytest.mark.parametrize("part", [2, 3])
def test_triangle_schedules_gather_each_entry_once_by_its_row(n, R, lanes, part):
    m = gen_mechanism(n, R)
    rp, ci = m.row_ptr, m.col_idx
    d = bcs.schedule_describe(rp, ci, lanes, part, bcs.BCS_SCHED_SPAN | bcs.BCS_SCHED_DIAG)
    rpl, seg, row, pos, col = d["rows_per_lane"], d["seg"], d["row"], d["pos"], d["col"]
    assert d["shape"] & bcs.BCS_SCHED_DIAG == 0
    starts = np.concatenate([[0], np.cumsum(seg)])
    owner = np.full((d["steps"], lanes), -1)
    for j in range(rpl):
        for lane in range(lanes):
            r = row[j, lane]
            if r == -2:
                owner[starts[1]:starts[2], lane] = row[0, lane]
            elif r >= 0:
                owner[starts[j]:starts[j + 1], lane] = r
    assert sorted(row[row >= 0].tolist()) == list(range(n))
    seen = {}
    for s in range(d["steps"]):
        for lane in range(lanes):
            p = int(pos[s, lane])
            if p >= 0:
                assert p not in seen
                seen[p] = (int(owner[s, lane]), int(col[s, lane]))
            else:
                assert col[s, lane] == n  # padding gathers the zero spare element
    want = {}
    for i in range(n):
        for k in range(rp[i], rp[i + 1]):
            if (ci[k] < i) if part == 2 else (ci[k] > i):
                want[k] = (i, int(ci[k]))
    assert seen == want


def test_program_needs_the_diagonal():
    rp = np.array([0, 2, 3, 5], np.int32)  # row 1 has no diagonal
    ci = np.array([0, 2, 0, 1, 2], np.int32)
    with pytest.raises(bcs.BcsError):
        bcs.ilu_describe(rp, ci, 16)
