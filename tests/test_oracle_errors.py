"""Error behaviour of the oracle on forced invalid inputs (no GPU)."""
import numpy as np
import pytest

import oracle as O
from paper_2401_03378_amd import workloads as W


def _base():
    return W.random_blocks(3, 6, 2, seed=0)


def _code(fn):
    try:
        fn()
    except O.OracleError as e:
        return e.code
    return 0


def test_valid_problem_is_accepted():
    assert O.validate(_base()) == 0


def _set(field, b, value):
    def f(p):
        p.blocks[field][b] = value(p) if callable(value) else value
    return f


def _link(b, value):
    def f(p):
        p.links["nbr"][b] = value
    return f


@pytest.mark.parametrize("mutate", [
    _set("offset", 1, lambda p: int(p.blocks["offset"][0]) + 5),   # overlap
    _set("offset", 0, -1),
    _set("offset", 2, lambda p: p.ncell),                          # out of range
    _set("ng", 0, 1),                                              # too few guards
    _link(0, [7, 9, -1, -1, -1, -1]),                              # no block 9
    _link(0, [-3, -1, -1, -1, -1, -1]),
])
def test_invalid_descriptors(mutate):
    p = _base()
    mutate(p)
    assert O.validate(p) == O.ORA_EINVAL
    assert _code(lambda: O.step(p, p.U0.copy())) == O.ORA_EINVAL


def test_mismatched_neighbour_faces():
    blocks, ncell = W.make_table([(6, 6, 6), (6, 4, 6)], 2, 3)
    links = np.zeros(2, dtype=W.LINK_DTYPE)
    links["nbr"] = [1, 1, -2, -2, -2, -2]
    p = W.random_blocks(3, 6, 2, seed=0)
    p.blocks, p.links, p.ncell = blocks, links, ncell
    assert O.validate(p) == O.ORA_EINVAL


def test_weno_needs_three_guards():
    p = W.random_blocks(3, 6, 2, seed=0, recon=W.WENO5, rk=3)
    assert O.validate(p) == O.ORA_EINVAL


def test_nonphysical_inputs():
    p = _base()
    m = W.interior_mask(p.blocks, p.ncell, 3)
    U = p.U0.copy()
    idx = np.flatnonzero(m)[17]
    U[4, idx] = -1.0                                      # negative energy -> p < 0
    assert _code(lambda: O.step(p, U)) == O.ORA_ENONPHYS
    U = p.U0.copy()
    U[0, np.flatnonzero(m)[3]] = np.nan
    assert _code(lambda: O.cfl_dt(p, U)) == O.ORA_ENONPHYS


def test_bad_dt():
    p = _base()
    U = p.U0.copy()
    assert _code(lambda: O.step(p, U, 0.0)) == O.ORA_EINVAL
    assert _code(lambda: O.step(p, U, -1e-3)) == O.ORA_EINVAL
