"""GPU tests of the context's state between calls: the launch lists that a
pass over every column keeps resident (they must follow nu, the system and
other column lists), and kernel error flags that a call reads back in stream
order with its one synchronisation (an error in pass 1 is reported as such,
and a later call on a valid system starts clean)."""
from __future__ import annotations

import numpy as np
import pytest

from gpu_helpers import gpu_context, log, np_, torch_cuda
import gen

pytestmark = pytest.mark.gpu


def _solve_state(ctx, s, nu):
    mu, E, A = ctx.solve(nu=nu, kT=s.kT, n_electrons=s.n_electrons)
    eps, w, nu_eff = (np_(x) for x in ctx.spectra())
    rho, pi = (np_(x) for x in ctx.density_matrix())
    return mu, E, A, eps, w, nu_eff, rho, pi


def _same(a, b):
    return all(np.array_equal(np.asarray(x), np.asarray(y)) for x, y in zip(a, b))


def test_resident_launch_lists_follow_nu_columns_and_system():
    """A context that alternates nu, runs a column subset in between (which
    replaces the resident lists) and is given its system again gives bitwise
    the results of fresh contexts (void cell: several cluster-size buckets)."""
    torch_cuda()
    s = gen.make("mini_void")
    ctx = gpu_context(s)
    first20 = _solve_state(ctx, s, 20)
    first30 = _solve_state(ctx, s, 30)
    again20 = _solve_state(ctx, s, 20)  # lists of nu = 30 resident: rebuilt
    cols = np.arange(0, 4 * s.n_atoms, 7, dtype=np.int32)
    ctx.column_spectra(cols, nu=20, kT=s.kT)  # other lists in the device buffers
    after_cols = _solve_state(ctx, s, 20)
    rowptr, colind, H, S = ctx._csr
    ctx.set_system(rowptr, colind, H, S, pos=ctx._pos, cell=s.cell, r_cluster=s.r_cluster)
    after_sys = _solve_state(ctx, s, 20)
    fresh20 = _solve_state(gpu_context(s), s, 20)
    ctx30 = gpu_context(s)
    fresh30 = _solve_state(ctx30, s, 30)
    log(f"[lists] mu20 {first20[0]!r} mu30 {first30[0]!r}")
    # the two contexts time their own launch plans and may keep different
    # ones (shape, workgroups per CU, cache size): the columns' bits do not
    # depend on that choice
    plan = lambda st: [(st["plan_threads"][b], st["plan_per_cu"][b], st["plan_cache"][b])  # noqa: E731
                       for b in range(len(st["plan_threads"])) if st["plan_threads"][b] > 0]
    log(f"[lists] plans (threads, per CU, cached blocks) {plan(ctx.stats())} | "
        f"{plan(ctx30.stats())}")
    assert _same(first20, fresh20)
    assert _same(first30, fresh30)
    assert _same(again20, fresh20)
    assert _same(after_cols, fresh20)
    assert _same(after_sys, fresh20)
    st = ctx.stats()
    assert st["krylov_buckets"] >= 2


def test_pass1_error_is_reported_and_the_next_system_starts_clean():
    """Clusters of one atom each leave every column's pattern row outside its
    cluster: pass 1 flags it, and the solve reports it as a pass-1 error after
    the chemical-potential kernels have run on the empty spectra.  With proper
    clusters again the same context solves to the bits of a fresh one."""
    torch = torch_cuda()
    from paper_1210_1531_amd import MagError, _lib as L
    s = gen.make("mini_vac")
    ctx = gpu_context(s)
    rowptr, colind, H, S = ctx._csr
    n = s.n_atoms
    self_ptr = torch.arange(n + 1, dtype=torch.int64, device="cuda")
    self_atoms = torch.arange(n, dtype=torch.int32, device="cuda")
    ctx.set_system(rowptr, colind, H, S, pos=ctx._pos, cell=s.cell, clus_ptr=self_ptr,
                   clus_atoms=self_atoms)
    with pytest.raises(MagError) as e:
        ctx.solve(nu=s.nu, kT=s.kT, n_electrons=s.n_electrons)
    log(f"[pass-1 error] status {e.value.status}: {e.value}")
    assert e.value.status == L.MAG_EINVAL
    assert "pass 1" in str(e.value) and "cluster" in str(e.value)
    ctx.set_system(rowptr, colind, H, S, pos=ctx._pos, cell=s.cell, r_cluster=s.r_cluster)
    got = _solve_state(ctx, s, s.nu)
    F = np_(ctx.forces(ctx._sk))
    ref_ctx = gpu_context(s)
    ref = _solve_state(ref_ctx, s, s.nu)
    Fref = np_(ref_ctx.forces(ref_ctx._sk))
    assert _same(got, ref)
    assert np.array_equal(F, Fref)


def test_columns_do_not_depend_on_the_block_cache(monkeypatch):
    """The fused SpMV reads a row's first blocks from the LDS cache and streams
    the rest; the two accumulator pairs take the blocks by their offset in the
    row, so a context whose plans hold no cache (every block streamed) gives
    the bits of one with the cache."""
    torch_cuda()
    s = gen.make("mini_vac")
    ref_ctx = gpu_context(s)
    ref = _solve_state(ref_ctx, s, s.nu)
    monkeypatch.setenv("MAG_LDS_CACHE", "0")  # read when a context makes its plans
    ctx = gpu_context(s)
    got = _solve_state(ctx, s, s.nu)
    cached = [c for c, t in zip(ref_ctx.stats()["plan_cache"], ref_ctx.stats()["plan_threads"])
              if t > 0]
    uncached = [c for c, t in zip(ctx.stats()["plan_cache"], ctx.stats()["plan_threads"]) if t > 0]
    log(f"[cache] cached blocks per plan {cached} against {uncached}")
    assert max(cached) > 0 and max(uncached) == 0
    assert _same(got, ref)
