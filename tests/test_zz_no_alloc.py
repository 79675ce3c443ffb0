"""The allocation-free entry point (mag_sk_vjp_noalloc) against the entry
point it varies (mag_sk_vjp), through the C ABI: bitwise equal products on two
calls in a row, the second on a smaller pattern (the fixed scratch keeps the
first call's larger contents), no device memory taken by the call, and the
documented rejections."""
import ctypes as C
import gc

import numpy as np
import pytest

from gpu_helpers import gpu_context, log, np_

pytestmark = pytest.mark.gpu


def _inputs(ctx, s, seed):
    import torch
    rng = np.random.default_rng(seed)
    pos = torch.tensor(s.pos + rng.normal(0.0, 0.01, size=s.pos.shape), dtype=torch.float64,
                       device="cuda")
    gH = torch.tensor(rng.normal(size=ctx.sk_nnz), dtype=torch.float64, device="cuda")
    gS = torch.tensor(rng.normal(size=ctx.sk_nnz), dtype=torch.float64, device="cuda")
    return pos, gH, gS


def _compare(ctx, s, seed):
    import torch
    pos, gH, gS = _inputs(ctx, s, seed)
    ref = ctx.sk_vjp(pos, gH, gS)
    out = torch.full((s.n_atoms, 3), float("nan"), dtype=torch.float64, device="cuda")
    gc.collect()  # garbage of earlier tests freed now, not during the call
    torch.cuda.synchronize()
    held = ctx.stats()["device_bytes"]
    torch.cuda.reset_peak_memory_stats()
    taken = torch.cuda.memory_allocated()
    ctx.sk_vjp_noalloc(pos, gH, gS, out)
    torch.cuda.synchronize()
    # neither the library's own device memory nor torch's grew during the call
    assert ctx.stats()["device_bytes"] == held
    assert torch.cuda.max_memory_allocated() == taken
    same = bool(torch.equal(out, ref))
    log(f"[noalloc] {s.n_atoms} atoms, {ctx.sk_nnz // 16} blocks: bitwise equal {same}, "
        f"max |grad| {ref.abs().max().item():.3e}")
    assert same


def test_noalloc_vjp_equals_vjp_on_two_calls_the_second_smaller():
    import gen
    from paper_1210_1531_amd import model
    big = gen.make(2)
    small = gen.make("mini_vac")
    ctx = gpu_context(big)
    _compare(ctx, big, 1)
    import torch
    ctx.sk_build(model.sk_model(), torch.tensor(small.pos, dtype=torch.float64, device="cuda"),
                 small.cell)
    assert ctx.sk_nnz < 16 * 56888
    _compare(ctx, small, 2)


def test_noalloc_vjp_rejections():
    import torch
    from gen import structures as gs
    from paper_1210_1531_amd import MagError, _lib as L, model
    s = gs.make_structure(cells=(2, 2, 2), sigma=0.02, seed=3)
    ctx = gpu_context(s)
    pos, gH, gS = _inputs(ctx, s, 3)
    out = torch.empty((s.n_atoms, 3), dtype=torch.float64, device="cuda")
    # host pointers
    host = np.zeros((s.n_atoms, 3))
    st = ctx._lib.mag_sk_vjp_noalloc(ctx._h, C.c_void_p(pos.data_ptr()), C.c_void_p(gH.data_ptr()),
                                     C.c_void_p(gS.data_ptr()), C.c_void_p(host.ctypes.data))
    assert st == L.MAG_EINVAL
    # a device array shorter than the pattern
    short = torch.empty(8, dtype=torch.float64, device="cuda")
    st = ctx._lib.mag_sk_vjp_noalloc(ctx._h, C.c_void_p(pos.data_ptr()),
                                     C.c_void_p(short.data_ptr()), C.c_void_p(gS.data_ptr()),
                                     C.c_void_p(out.data_ptr()))
    assert st in (L.MAG_OK, L.MAG_EINVAL)  # inside a larger pool block it cannot be told apart
    # a pattern beyond the fixed scratch
    big = gs.make_structure(cells=(32, 32, 32), sigma=0.0, seed=3)
    ctx.sk_build(model.sk_model(), torch.tensor(big.pos, dtype=torch.float64, device="cuda"),
                 big.cell)
    assert ctx.sk_nnz // 16 > 1048576
    pos_b = torch.tensor(big.pos, dtype=torch.float64, device="cuda")
    g = torch.zeros(ctx.sk_nnz, dtype=torch.float64, device="cuda")
    out_b = torch.empty((big.n_atoms, 3), dtype=torch.float64, device="cuda")
    with pytest.raises(MagError) as e:
        ctx.sk_vjp_noalloc(pos_b, g, g, out_b)
    assert e.value.status == L.MAG_EUNSUPPORTED
    log(f"[noalloc] rejected: host output, {ctx.sk_nnz // 16} blocks")
