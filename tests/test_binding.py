"""The Python binding against a stub of the C library (no GPU): every method
passes the argument count and types that include/mag.h declares."""
import ctypes as C

import numpy as np
import pytest

from paper_1210_1531_amd import _lib as L
from paper_1210_1531_amd import mag as M
from paper_1210_1531_amd import model


class _Stub:
    """Records calls; checks arity against the prototypes; returns MAG_OK."""

    def __init__(self):
        self.calls = []

    def __getattr__(self, name):
        res, argtypes = L.PROTOTYPES[name]

        def fn(*args):
            assert len(args) == len(argtypes), (name, len(args), len(argtypes))
            for a, t in zip(args, argtypes):
                if t is C.c_void_p:
                    assert a is None or isinstance(a, (C.c_void_p, int)), (name, a)
            self.calls.append(name)
            if name == "mag_last_error":
                return b""
            if name == "mag_get_clusters" and args[3] is not None:
                args[3]._obj.value = 10
            return 0 if res is not None else None
        return fn


@pytest.fixture()
def ctx(monkeypatch):
    c = M.Context.__new__(M.Context)
    c._lib = _Stub()
    c._h = C.c_void_p(1)
    c.device = 0
    c.device_outputs = False
    c.n_atoms = 4
    c.nnz = 256
    c.sk_n = 4
    c.sk_nnz = 256
    c.opts = M.make_opts(nu=8, kT=0.1, n_electrons=16)
    yield c
    c._h = None


def test_every_method_matches_the_prototypes(ctx, monkeypatch):
    monkeypatch.setattr(L, "load", lambda: _Stub())
    pos = np.zeros((4, 3))
    cell = (10.0, 10.0, 10.0)
    ctx.sk_build(model.sk_model(), pos, cell)
    ctx.sk_get_csr()
    ctx.sk_values(pos)
    ctx.sk_vjp(pos, np.zeros(ctx.sk_nnz), np.zeros(ctx.sk_nnz))
    with pytest.raises(ValueError):  # device tensors only: it allocates nothing for the caller
        ctx.sk_vjp_noalloc(pos, np.zeros(ctx.sk_nnz), np.zeros(ctx.sk_nnz), np.zeros((4, 3)))
    rowptr = np.arange(17, dtype=np.int64) * 16
    ctx.set_system(rowptr, np.zeros(256, np.int32), np.zeros(256), np.zeros(256), pos=pos,
                   cell=cell, r_cluster=6.0)
    ctx.update_values(np.zeros(256), np.zeros(256))
    ctx.get_clusters()
    ctx.solve(nu=8, kT=0.1, n_electrons=16.0)
    ctx.spectra()
    ctx.energy()
    ctx.column_spectra([0, 1], nu=8, kT=0.1)
    ctx.density_matrix()
    ctx.cluster_columns([0, 3])
    ctx.green_columns([0], [0.5 + 0.1j], nu=8, kT=0.1)
    ctx.backward(1.0)
    ctx.forces(model.sk_model())
    ctx.forces_exact(model.sk_model())
    ctx.icohp(model.sk_model())
    ctx.cohp([0.0, 1.0], 0.1)
    ctx.cocg_columns([0, 1], [0.5 + 0.1j])
    ctx.pair_repulsion(13.18, 4.0)
    ctx.md_run(model.sk_model(), pos, np.zeros((4, 3)), cell, 0.5, 12.011, 2, phi0=13.18,
               r_cluster=6.0, nu=8, kT=0.1, n_electrons=16.0)
    ctx.stats()
    called = set(ctx._lib.calls)
    # the allocation-free entry point takes device tensors only; its call
    # through the C ABI is covered by the GPU test that runs last
    expected = set(L.PROTOTYPES) - {"mag_create", "mag_destroy", "mag_version", "mag_opts_default",
                                    "mag_last_error", "mag_sk_vjp_noalloc"}
    assert expected <= called, expected - called
