"""The tree solve without allocation against the allocating one, through the
C ABI: bitwise equal results on two calls in a row (the second smaller),
both equal to the oracle's elimination on every cell."""
import ctypes as C

import numpy as np
import pytest

import oracle
from paper_2411_16445_amd import binding as B

pytestmark = pytest.mark.gpu


def _random_trees(rng, n_cells, max_cv):
    """Random trees (one-row cells included) with diagonally dominant
    symmetric systems: cell-local parents, diagonal, couplings, rhs."""
    sizes = rng.integers(1, max_cv + 1, n_cells)
    sizes[0] = 1
    cv_off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    parent = np.empty(cv_off[-1], np.int32)
    for k in range(n_cells):
        n = sizes[k]
        parent[cv_off[k]] = -1
        if n > 1:
            # mostly chains with random branch points
            loc = np.arange(1, n)
            p = loc - 1
            jump = rng.random(n - 1) < 0.3
            p[jump] = (rng.random(jump.sum()) * loc[jump]).astype(np.int64)
            parent[cv_off[k] + 1:cv_off[k + 1]] = p
    n_cv = int(cv_off[-1])
    off = -rng.uniform(0.1, 50.0, n_cv)
    diag = np.zeros(n_cv)
    for k in range(n_cells):
        a = cv_off[k]
        for i in range(1, sizes[k]):
            diag[a + i] += -off[a + i]
            diag[a + parent[a + i]] += -off[a + i]
    diag += rng.uniform(0.01, 5.0, n_cv)
    rhs = rng.normal(0.0, 10.0, n_cv)
    return cv_off, parent, diag, off, rhs


def _oracle_solve(cv_off, parent, diag, off, rhs):
    x = np.empty_like(diag)
    for k in range(len(cv_off) - 1):
        a, b = cv_off[k], cv_off[k + 1]
        x[a:b] = oracle.hines(parent[a:b].astype(np.int64), off[a:b], diag[a:b], rhs[a:b])
    return x


def _solve(fn, case, stream):
    import torch
    cv_off, parent, diag, off, rhs = case
    dev = [torch.from_numpy(a).cuda() for a in (cv_off, parent, diag, off, rhs)]
    x = torch.full((len(diag),), -7.0, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    st = fn(len(cv_off) - 1, len(diag), *[C.c_void_p(t.data_ptr()) for t in dev],
            C.c_void_p(x.data_ptr()), C.c_void_p(stream))
    assert st == B.PA_OK, st
    torch.cuda.synchronize()
    return x.cpu().numpy()


def test_tree_solve_without_allocation_matches_allocating_solve():
    import torch
    lib = B.load_library()
    stream = torch.cuda.current_stream().cuda_stream
    rng = np.random.default_rng(20)
    for n_cells, max_cv in ((3000, 300), (257, 40)):   # second call smaller
        print(f"[case] tree solve {n_cells} cells up to {max_cv} rows", flush=True)
        case = _random_trees(rng, n_cells, max_cv)
        want = _oracle_solve(*case)
        x_alloc = _solve(lib.pa_tree_solve, case, stream)
        x_noalloc = _solve(lib.pa_tree_solve_noalloc, case, stream)
        np.testing.assert_array_equal(x_noalloc, x_alloc)
        np.testing.assert_allclose(x_alloc, want, rtol=1e-12, atol=1e-12 * np.abs(want).max())


def test_tree_solve_without_allocation_rejects_oversize_and_flags_bad_trees():
    import torch
    lib = B.load_library()
    stream = torch.cuda.current_stream().cuda_stream
    z = torch.zeros(4, dtype=torch.float64, device="cuda")
    zi = torch.zeros(4, dtype=torch.int64, device="cuda")
    p = C.c_void_p
    st = lib.pa_tree_solve_noalloc(1, (1 << 20) + 1, p(zi.data_ptr()), p(zi.data_ptr()), p(z.data_ptr()),
                                   p(z.data_ptr()), p(z.data_ptr()), p(z.data_ptr()), p(stream))
    assert st == B.PA_ERANGE
    # a parent pointing forward: the cell's rows are NaN, the other cell solves
    cv_off = np.array([0, 3, 5], np.int64)
    parent = np.array([-1, 2, 0, -1, 0], np.int32)
    diag = np.full(5, 4.0)
    off = np.full(5, -1.0)
    rhs = np.arange(5.0)
    x = _solve(lib.pa_tree_solve_noalloc, (cv_off, parent, diag, off, rhs), stream)
    assert np.isnan(x[:3]).all()
    np.testing.assert_allclose(x[3:], oracle.hines(np.array([-1, 0]), off[3:], diag[3:], rhs[3:]), rtol=1e-15)
