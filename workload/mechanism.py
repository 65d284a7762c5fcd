"""Random mass-action mechanisms and per-cell linear-system inputs.

Chemistry background (Section 2.2, the displayed rate equations): each species
concentration y_i changes at the rate f_i = sum over reactions j of the
reaction's contribution, and in the multi-cell form y_ik is species i of cell
k.  A mechanism here is a list of elementary reactions

    unimolecular  A -> B             rate w = k * y_A
    bimolecular   A + B -> C + D     rate w = k * y_A * y_B   (A == B allowed)

with f = S w (S = stoichiometry, products minus reactants) and the Jacobian
J = df/dy.  Two structural choices make useful invariants:

* every reaction keeps the molecule count (1 -> 1, 2 -> 2), so every column of
  S sums to zero and therefore every column of J sums to zero;
* no product is also a reactant, so each diagonal entry of J is <= 0.

Because f is at most quadratic in y, a central difference of f reproduces a
column of J exactly up to rounding; the tests use that to check J.

The Jacobian sparsity pattern (shared by all cells) is the union, over
reactions, of (i, j) with i any species of the reaction and j one of its
reactants, plus the full diagonal, stored as sorted CSR (int32).

All random draws go through ``numpy.random.Generator(PCG64(seed))`` in a fixed
order so that the same seed gives the same bits everywhere.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Tuple

import numpy as np

# Probability that a reaction is unimolecular.
P_UNI = 1.0 / 3.0
# Rate constants are log-uniform on [1e-12, 1e2].
LOG10_K_RANGE = (-12.0, 2.0)
# Concentrations are log-uniform on [1e-6, 1e3].
LOG10_Y_RANGE = (-6.0, 3.0)
# Step sizes h are log-uniform on [1e-3, h_max]; gamma = 0.5 * h.
LOG10_H_MIN = -3.0


def mech_seed(n: int) -> int:
    """Seed of the mechanism with ``n`` species (24050000 + n)."""
    return 24050000 + n


def cell_seed(config: int) -> int:
    """Seed of the per-cell draws of workload configuration ``config`` (1-based)."""
    return 1736300 + config


@dataclasses.dataclass
class Mechanism:
    n: int
    reactants: np.ndarray  # [R, 2] int64, second entry -1 for unimolecular
    products: np.ndarray   # [R, 2] int64, second entry -1 for unimolecular
    k: np.ndarray          # [R] float64 rate constants
    row_ptr: np.ndarray    # [n + 1] int32
    col_idx: np.ndarray    # [nnz] int32
    # Derivative terms of J in a fixed order: J[:, pos] += coef * (y[:, yidx] or 1)
    term_pos: np.ndarray   # [T] int64
    term_coef: np.ndarray  # [T] float64
    term_y: np.ndarray     # [T] int64, -1 = no concentration factor

    @property
    def nnz(self) -> int:
        return int(self.col_idx.shape[0])

    @property
    def R(self) -> int:
        return int(self.k.shape[0])

    def diag_pos(self) -> np.ndarray:
        """CSR position of each diagonal entry."""
        out = np.empty(self.n, dtype=np.int64)
        for i in range(self.n):
            lo, hi = self.row_ptr[i], self.row_ptr[i + 1]
            hit = np.nonzero(self.col_idx[lo:hi] == i)[0]
            out[i] = lo + int(hit[0])
        return out

    def dense_pattern(self) -> np.ndarray:
        m = np.zeros((self.n, self.n), dtype=bool)
        for i in range(self.n):
            m[i, self.col_idx[self.row_ptr[i]:self.row_ptr[i + 1]]] = True
        return m


def _species(reac: np.ndarray, prod: np.ndarray) -> List[int]:
    out = []
    for s in list(reac) + list(prod):
        if s >= 0 and s not in out:
            out.append(int(s))
    return out


def _stoich(reac: np.ndarray, prod: np.ndarray) -> Dict[int, int]:
    st: Dict[int, int] = {}
    for s in reac:
        if s >= 0:
            st[int(s)] = st.get(int(s), 0) - 1
    for s in prod:
        if s >= 0:
            st[int(s)] = st.get(int(s), 0) + 1
    return st


def gen_mechanism(n: int, R: int, seed: int | None = None, p_uni: float = P_UNI) -> Mechanism:
    """Draw a conserving, non-autocatalytic mass-action mechanism.

    Per reaction, in this order: u ~ U(0,1) decides uni (u < p_uni) or bi;
    uni: A uniform over species, B uniform over species != A;
    bi: A, B uniform over species (A == B allowed), C, D uniform over species
    not in {A, B} (C == D allowed).  Then all R rate constants
    k = 10**U(-12, 2) are drawn at once.
    """
    if n < 3:
        raise ValueError("a mechanism needs at least 3 species")
    rng = np.random.Generator(np.random.PCG64(mech_seed(n) if seed is None else seed))
    reac = np.full((R, 2), -1, dtype=np.int64)
    prod = np.full((R, 2), -1, dtype=np.int64)
    for r in range(R):
        if rng.uniform() < p_uni:
            a = int(rng.integers(n))
            b = int(rng.integers(n - 1))
            if b >= a:
                b += 1
            reac[r, 0] = a
            prod[r, 0] = b
        else:
            a = int(rng.integers(n))
            b = int(rng.integers(n))
            excl = sorted({a, b})
            pool = np.array([s for s in range(n) if s not in excl], dtype=np.int64)
            c = int(pool[rng.integers(pool.shape[0])])
            d = int(pool[rng.integers(pool.shape[0])])
            reac[r] = (a, b)
            prod[r] = (c, d)
    k = 10.0 ** rng.uniform(LOG10_K_RANGE[0], LOG10_K_RANGE[1], size=R)

    # Pattern: species of the reaction x reactants of the reaction, plus diagonal.
    entries = set((i, i) for i in range(n))
    for r in range(R):
        sp = _species(reac[r], prod[r])
        for j in reac[r]:
            if j >= 0:
                for i in sp:
                    entries.add((i, int(j)))
    rows: List[List[int]] = [[] for _ in range(n)]
    for (i, j) in entries:
        rows[i].append(j)
    row_ptr = np.zeros(n + 1, dtype=np.int32)
    cols: List[int] = []
    for i in range(n):
        rj = sorted(rows[i])
        cols.extend(rj)
        row_ptr[i + 1] = len(cols)
    col_idx = np.asarray(cols, dtype=np.int32)
    pos_of: Dict[Tuple[int, int], int] = {}
    for i in range(n):
        for p in range(row_ptr[i], row_ptr[i + 1]):
            pos_of[(i, int(col_idx[p]))] = p

    # Derivative terms d f_i / d y_j = S_ir * d w_r / d y_j, in reaction order.
    t_pos: List[int] = []
    t_coef: List[float] = []
    t_y: List[int] = []
    for r in range(R):
        st = _stoich(reac[r], prod[r])
        a, b = int(reac[r, 0]), int(reac[r, 1])
        if b < 0:  # w = k y_a
            derivs = [(a, 1.0, -1)]
        elif a == b:  # w = k y_a^2
            derivs = [(a, 2.0, a)]
        else:  # w = k y_a y_b
            derivs = [(a, 1.0, b), (b, 1.0, a)]
        for (j, mult, yfac) in derivs:
            for i, s in st.items():
                t_pos.append(pos_of[(i, j)])
                t_coef.append(float(s) * mult * float(k[r]))
                t_y.append(yfac)
    return Mechanism(
        n=n, reactants=reac, products=prod, k=k, row_ptr=row_ptr, col_idx=col_idx,
        term_pos=np.asarray(t_pos, dtype=np.int64),
        term_coef=np.asarray(t_coef, dtype=np.float64),
        term_y=np.asarray(t_y, dtype=np.int64),
    )


def rates(mech: Mechanism, y: np.ndarray) -> np.ndarray:
    """f(y) = S w(y) for concentrations ``y`` of shape [..., n]."""
    y = np.asarray(y, dtype=np.float64)
    f = np.zeros_like(y)
    for r in range(mech.R):
        a, b = int(mech.reactants[r, 0]), int(mech.reactants[r, 1])
        w = mech.k[r] * y[..., a]
        if b >= 0:
            w = w * y[..., b]
        for i, s in _stoich(mech.reactants[r], mech.products[r]).items():
            f[..., i] += s * w
    return f


def jacobian_values(mech: Mechanism, y: np.ndarray) -> np.ndarray:
    """J = df/dy on the mechanism's pattern: [C, n] concentrations -> [C, nnz]."""
    y = np.atleast_2d(np.asarray(y, dtype=np.float64))
    J = np.zeros((y.shape[0], mech.nnz), dtype=np.float64)
    for pos, coef, yi in zip(mech.term_pos, mech.term_coef, mech.term_y):
        if yi < 0:
            J[:, pos] += coef
        else:
            J[:, pos] += coef * y[:, yi]
    return J


def gen_cells(mech: Mechanism, ncells: int, seed: int, h_max: float = 10.0,
              mode: str = "realistic") -> Dict[str, np.ndarray]:
    """Per-cell inputs of the batched system (I - gamma*J) x = b.

    Draw order: y [C, n] = 10**U(-6, 3); h [C] = 10**U(-3, log10 h_max);
    b [C, n] ~ N(0, 1).  gamma = 0.5 * h.  ``mode="ideal"`` copies cell 0 into
    every cell (the ideal case of Section 4.2: identical initial conditions).
    Returns float64 arrays ``values`` [C, nnz] (= J), ``gamma`` [C], ``b`` [C, n]
    and ``y`` [C, n].
    """
    if mode not in ("realistic", "ideal"):
        raise ValueError("mode must be 'realistic' or 'ideal'")
    rng = np.random.Generator(np.random.PCG64(seed))
    n = mech.n
    y = 10.0 ** rng.uniform(LOG10_Y_RANGE[0], LOG10_Y_RANGE[1], size=(ncells, n))
    h = 10.0 ** rng.uniform(LOG10_H_MIN, math.log10(h_max), size=ncells)
    b = rng.standard_normal(size=(ncells, n))
    if mode == "ideal" and ncells > 0:
        y[:] = y[0]
        h[:] = h[0]
        b[:] = b[0]
    values = jacobian_values(mech, y) if ncells > 0 else np.zeros((0, mech.nnz))
    return {"values": np.ascontiguousarray(values), "gamma": 0.5 * h,
            "b": np.ascontiguousarray(b), "y": y}


# The five workload configurations (sizes and ranges of the benchmark suite).
CONFIGS = {
    1: dict(mechs=[(80, 150)], ncells=[100], h_max=10.0),
    2: dict(mechs=[(80, 150)], ncells=[10_000], h_max=10.0),
    3: dict(mechs=[(80, 150)], ncells=[100_000], h_max=100.0),
    4: dict(mechs=[(30, 50), (80, 150), (200, 400)], ncells=[12_500, 25_000, 12_500], h_max=10.0),
    5: dict(mechs=[(80, 150)], ncells=[10_000], h_max=10.0),
}


def config_inputs(config: int, ncells: int | None = None, mode: str = "realistic"):
    """Mechanisms and cells of a configuration: list of (Mechanism, cells dict).

    ``ncells`` overrides the cell count of a single-mechanism configuration
    (the first ``ncells`` cells drawn from the configuration's seed are NOT the
    same as a prefix of the full draw; use it only for reduced-size runs).
    For configuration 5 the cells dict also carries the loss weights ``w``
    [C, n] ~ N(0, 1) drawn from seed cell_seed(5) + 1.
    """
    cfg = CONFIGS[config]
    out = []
    for m_i, ((n, R), C) in enumerate(zip(cfg["mechs"], cfg["ncells"])):
        if ncells is not None:
            C = ncells if len(cfg["mechs"]) == 1 else max(1, (ncells * C) // sum(cfg["ncells"]))
        mech = gen_mechanism(n, R)
        cells = gen_cells(mech, C, cell_seed(config) + 100 * m_i, h_max=cfg["h_max"], mode=mode)
        if config == 5:
            rng = np.random.Generator(np.random.PCG64(cell_seed(5) + 1))
            cells["w"] = rng.standard_normal(size=(C, n))
        out.append((mech, cells))
    return out
