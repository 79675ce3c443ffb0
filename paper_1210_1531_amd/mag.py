"""Python binding of libmag (argument marshalling only; all work runs in HIP).

Arrays may be NumPy arrays (host) or torch tensors on the GPU (device); each
call passes all of its arrays with one memory kind, moving host arrays to the
device when any argument already lives there.  Outputs are torch tensors on
the context's device when ``device_outputs`` is set, NumPy arrays otherwise.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import _lib as L

try:  # torch is plumbing only: device memory and the stream
    import torch
except Exception:  # pragma: no cover - torch is present in the supported image
    torch = None


class MagError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{L.STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


_WORKFLOWS = {"recompute": L.MAG_WORKFLOW_RECOMPUTE, "store": L.MAG_WORKFLOW_STORE,
              "auto": L.MAG_WORKFLOW_AUTO}
_SCHEDULES = {"auto": L.MAG_SCHED_AUTO, "persistent": L.MAG_SCHED_PERSISTENT,
              "grid": L.MAG_SCHED_GRID, "plain": L.MAG_SCHED_PLAIN,
              "graph": L.MAG_SCHED_GRAPH}

_NP = {np.float64: (torch.float64 if torch else None), np.int32: (torch.int32 if torch else None),
       np.int64: (torch.int64 if torch else None)}


def _is_dev(x):
    return torch is not None and isinstance(x, torch.Tensor) and x.is_cuda


def make_opts(nu=30, kT=0.1, n_electrons=0.0, mu_tol=1e-12, mu_fixed=None, breakdown=1e-12,
              workflow="auto", schedule="auto", eig_sweeps=0, keep_exact=False) -> L.MagOpts:
    o = L.MagOpts()
    L.load().mag_opts_default(C.byref(o))
    o.nu = int(nu)
    o.kT = float(kT)
    o.n_electrons = float(n_electrons)
    o.mu_tol = float(mu_tol)
    o.mu_fixed = float("nan") if mu_fixed is None else float(mu_fixed)
    o.breakdown = float(breakdown)
    o.workflow = _WORKFLOWS[workflow] if isinstance(workflow, str) else int(workflow)
    o.schedule = _SCHEDULES[schedule] if isinstance(schedule, str) else int(schedule)
    o.eig_sweeps = int(eig_sweeps)
    o.keep_exact = int(bool(keep_exact))
    return o


class Context:
    """One libmag context on one GPU."""

    def __init__(self, device: int = 0, device_outputs: bool = True, use_torch_stream: bool = True):
        self._lib = L.load()
        self.device = device
        self.device_outputs = bool(device_outputs and torch is not None and torch.cuda.is_available())
        stream = None
        if use_torch_stream and torch is not None and torch.cuda.is_available():
            stream = C.c_void_p(torch.cuda.current_stream(device).cuda_stream)
        h = C.c_void_p()
        st = self._lib.mag_create(C.byref(h), int(device), stream)
        if st != L.MAG_OK:
            raise MagError(st, "mag_create failed")
        self._h = h
        self.n_atoms = 0
        self.nnz = 0
        self.sk_n = 0
        self.sk_nnz = 0
        self.opts = None

    # ---------------------------------------------------------------- utils
    def close(self):
        if getattr(self, "_h", None):
            self._lib.mag_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, status):
        if status != L.MAG_OK:
            msg = self._lib.mag_last_error(self._h)
            raise MagError(status, msg.decode() if msg else "")

    def _torch_dev(self):
        return torch.device("cuda", self.device)

    def _inputs(self, arrays, dtypes):
        """Pointers and memory kind for a set of input arrays (None allowed)."""
        dev = any(_is_dev(a) for a in arrays if a is not None)
        keep, ptrs = [], []
        for a, dt in zip(arrays, dtypes):
            if a is None:
                ptrs.append(None)
                continue
            if dev:
                t = a if _is_dev(a) else torch.as_tensor(np.asarray(a))
                t = t.to(device=self._torch_dev(), dtype=_NP[dt]).contiguous()
                keep.append(t)
                ptrs.append(C.c_void_p(t.data_ptr()))
            else:
                x = np.ascontiguousarray(np.asarray(a), dtype=dt)
                keep.append(x)
                ptrs.append(C.c_void_p(x.ctypes.data))
        return ptrs, (L.MAG_DEVICE if dev else L.MAG_HOST), keep

    def _outputs(self, shapes_dtypes):
        outs, ptrs = [], []
        for shape, dt in shapes_dtypes:
            if self.device_outputs:
                t = torch.empty(shape, dtype=_NP[dt], device=self._torch_dev())
                outs.append(t)
                ptrs.append(C.c_void_p(t.data_ptr()))
            else:
                x = np.empty(shape, dtype=dt)
                outs.append(x)
                ptrs.append(C.c_void_p(x.ctypes.data))
        kind = L.MAG_DEVICE if self.device_outputs else L.MAG_HOST
        return outs, ptrs, kind

    # -------------------------------------------------------- Slater-Koster
    def sk_build(self, model, pos, cell):
        """Pattern and values of H, S from positions (A0); returns nnz."""
        pos_np = pos
        ptrs, kind, _keep = self._inputs([pos_np], [np.float64])
        n = int(pos.shape[0])
        cellv = (C.c_double * 3)(*[float(x) for x in cell])
        nnz = C.c_int64()
        self._check(self._lib.mag_sk_build(self._h, C.byref(model), n, ptrs[0], cellv, kind,
                                           C.byref(nnz)))
        self.sk_n = n
        self.sk_nnz = int(nnz.value)
        return self.sk_nnz

    def sk_get_csr(self):
        m = 4 * self.sk_n
        rowptr, colind, H, S = self._outputs_call(
            self._lib.mag_sk_get_csr,
            [((m + 1,), np.int64), ((self.sk_nnz,), np.int32), ((self.sk_nnz,), np.float64),
             ((self.sk_nnz,), np.float64)])
        return rowptr, colind, H, S

    def _outputs_call(self, fn, shapes_dtypes, *before):
        outs, ptrs, kind = self._outputs(shapes_dtypes)
        self._check(fn(self._h, *before, *ptrs, kind))
        return outs

    def sk_values(self, pos):
        ptrs, kind, _k = self._inputs([pos], [np.float64])
        outs, optrs, okind = self._outputs([((self.sk_nnz,), np.float64)] * 2)
        if kind != okind:
            ptrs, kind, _k = self._inputs([self._as_kind(pos, okind)], [np.float64])
        self._check(self._lib.mag_sk_values(self._h, ptrs[0], optrs[0], optrs[1], okind))
        return outs[0], outs[1]

    def _as_kind(self, a, kind):
        if kind == L.MAG_DEVICE:
            return a if _is_dev(a) else torch.as_tensor(np.asarray(a), device=self._torch_dev())
        return a.detach().cpu().numpy() if torch is not None and isinstance(a, torch.Tensor) else a

    def sk_vjp(self, pos, gH, gS):
        outs, optrs, okind = self._outputs([((self.sk_n, 3), np.float64)])
        ptrs, kind, _k = self._inputs([self._as_kind(pos, okind), self._as_kind(gH, okind),
                                       self._as_kind(gS, okind)], [np.float64] * 3)
        self._check(self._lib.mag_sk_vjp(self._h, ptrs[0], ptrs[1], ptrs[2], optrs[0], okind))
        return outs[0]

    def sk_vjp_noalloc(self, pos, gH, gS, out):
        """sk_vjp without any device allocation (mag_sk_vjp_noalloc): every
        argument is a contiguous float64 tensor on the context's device, and
        the product is written into `out` (n_atoms x 3), which is returned."""
        for x in (pos, gH, gS, out):
            if not (_is_dev(x) and x.dtype == torch.float64 and x.is_contiguous()):
                raise ValueError("sk_vjp_noalloc takes contiguous float64 device tensors")
        self._check(self._lib.mag_sk_vjp_noalloc(self._h, C.c_void_p(pos.data_ptr()),
                                                 C.c_void_p(gH.data_ptr()),
                                                 C.c_void_p(gS.data_ptr()),
                                                 C.c_void_p(out.data_ptr())))
        return out

    # --------------------------------------------------------------- system
    def set_system(self, rowptr, colind, H, S, pos=None, cell=(0.0, 0.0, 0.0), r_cluster=0.0,
                   clus_ptr=None, clus_atoms=None):
        arrays = [rowptr, colind, H, S, pos, clus_ptr, clus_atoms]
        dts = [np.int64, np.int32, np.float64, np.float64, np.float64, np.int64, np.int32]
        ptrs, kind, _keep = self._inputs(arrays, dts)
        s = L.MagSystem()
        s.n_atoms = (len(rowptr) - 1) // 4
        s.nnz = len(colind)
        s.rowptr, s.colind, s.H, s.S, s.pos, s.clus_ptr, s.clus_atoms = [
            (p.value if p is not None else None) for p in ptrs]
        for d in range(3):
            s.cell[d] = float(cell[d])
        s.r_cluster = float(r_cluster)
        self._check(self._lib.mag_set_system(self._h, C.byref(s), kind))
        self.n_atoms = int(s.n_atoms)
        self.nnz = int(s.nnz)

    def update_values(self, H, S):
        ptrs, kind, _keep = self._inputs([H, S], [np.float64, np.float64])
        self._check(self._lib.mag_update_values(self._h, ptrs[0], ptrs[1], kind))

    def get_clusters(self):
        total = C.c_int64()
        self._check(self._lib.mag_get_clusters(self._h, None, None, C.byref(total), L.MAG_HOST))
        outs, ptrs, kind = self._outputs([((self.n_atoms + 1,), np.int64),
                                          ((total.value,), np.int32)])
        self._check(self._lib.mag_get_clusters(self._h, ptrs[0], ptrs[1], None, kind))
        return outs

    # ---------------------------------------------------------------- solve
    @property
    def M(self):
        return 4 * self.n_atoms

    def solve(self, **kw):
        """Pass 1 + mu + energies; returns (mu, E_band, A_free)."""
        o = make_opts(**kw)
        mu, E, A = C.c_double(), C.c_double(), C.c_double()
        self._check(self._lib.mag_solve_columns(self._h, C.byref(o), C.byref(mu), C.byref(E),
                                                C.byref(A)))
        self.opts = o
        return mu.value, E.value, A.value

    def spectra(self):
        nu = self.opts.nu
        return self._outputs_call(self._lib.mag_spectra, [((self.M, nu), np.float64),
                                                          ((self.M, nu), np.float64),
                                                          ((self.M,), np.int32)])

    def energy(self):
        v = [C.c_double() for _ in range(4)]
        self._check(self._lib.mag_energy(self._h, *[C.byref(x) for x in v]))
        return dict(E_band=v[0].value, A_free=v[1].value, N=v[2].value, S_ent=v[3].value)

    def column_spectra(self, cols, **kw):
        o = make_opts(**kw)
        cols = np.ascontiguousarray(np.asarray(cols, dtype=np.int32))
        n = cols.size
        outs, ptrs, kind = self._outputs([((n, o.nu), np.float64), ((n, o.nu), np.float64),
                                          ((n,), np.int32)])
        cp, ck, _k = self._inputs([self._as_kind(cols, kind)], [np.int32])
        self._check(self._lib.mag_column_spectra(self._h, C.byref(o), cp[0], n, *ptrs, kind))
        return outs

    def density_matrix(self):
        return self._outputs_call(self._lib.mag_density_matrix,
                                  [((self.nnz,), np.float64), ((self.nnz,), np.float64)])

    def cluster_columns(self, cols):
        cols = np.ascontiguousarray(np.asarray(cols, dtype=np.int32))
        n = cols.size
        off = np.zeros(n + 1, dtype=np.int64)
        self._check(self._lib.mag_cluster_columns(self._h, C.c_void_p(cols.ctypes.data), n, None,
                                                  C.c_void_p(off.ctypes.data), L.MAG_HOST))
        outs, ptrs, kind = self._outputs([((int(off[-1]),), np.float64)])
        cp, _ck, _k = self._inputs([self._as_kind(cols, kind)], [np.int32])
        self._check(self._lib.mag_cluster_columns(self._h, cp[0], n, ptrs[0],
                                                  C.c_void_p(off.ctypes.data), kind))
        return outs[0], off

    def green_columns(self, cols, z, **kw):
        o = make_opts(**kw)
        cols = np.ascontiguousarray(np.asarray(cols, dtype=np.int32))
        z = np.ascontiguousarray(np.asarray(z, dtype=np.complex128).ravel())
        zz = np.ascontiguousarray(np.stack([z.real, z.imag], axis=1).ravel())
        n, nz = cols.size, z.size
        off = np.zeros(n + 1, dtype=np.int64)
        self._check(self._lib.mag_green_columns(self._h, C.byref(o), C.c_void_p(cols.ctypes.data),
                                                n, C.c_void_p(zz.ctypes.data), nz, None,
                                                C.c_void_p(off.ctypes.data), L.MAG_HOST))
        out = np.empty(2 * int(off[-1]) * nz, dtype=np.float64)
        self._check(self._lib.mag_green_columns(self._h, C.byref(o), C.c_void_p(cols.ctypes.data),
                                                n, C.c_void_p(zz.ctypes.data), nz,
                                                C.c_void_p(out.ctypes.data),
                                                C.c_void_p(off.ctypes.data), L.MAG_HOST))
        return out[0::2] + 1j * out[1::2], off

    def cocg_columns(self, cols, z, tol=1e-10, max_iter=2000):
        """Columns of (z S_C - H_C)^-1 by COCG on each column's cluster (see
        mag_cocg_columns).  Returns (G, offsets, iters): G complex in the layout
        of green_columns, iters (n, nz) steps taken or -1."""
        cols = np.ascontiguousarray(np.asarray(cols, dtype=np.int32))
        z = np.ascontiguousarray(np.asarray(z, dtype=np.complex128).ravel())
        zz = np.ascontiguousarray(np.stack([z.real, z.imag], axis=1).ravel())
        n, nz = cols.size, z.size
        off = np.zeros(n + 1, dtype=np.int64)
        self._check(self._lib.mag_cocg_columns(self._h, C.c_void_p(cols.ctypes.data), n,
                                               C.c_void_p(zz.ctypes.data), nz, float(tol),
                                               int(max_iter), None, C.c_void_p(off.ctypes.data),
                                               None, L.MAG_HOST))
        out = np.empty(2 * int(off[-1]) * nz, dtype=np.float64)
        iters = np.empty((n, nz), dtype=np.int32)
        self._check(self._lib.mag_cocg_columns(self._h, C.c_void_p(cols.ctypes.data), n,
                                               C.c_void_p(zz.ctypes.data), nz, float(tol),
                                               int(max_iter), C.c_void_p(out.ctypes.data),
                                               C.c_void_p(off.ctypes.data),
                                               C.c_void_p(iters.ctypes.data), L.MAG_HOST))
        return out[0::2] + 1j * out[1::2], off, iters

    def backward(self, gA=1.0):
        outs, ptrs, kind = self._outputs([((self.nnz,), np.float64), ((self.nnz,), np.float64)])
        self._check(self._lib.mag_backward(self._h, float(gA), ptrs[0], ptrs[1], kind))
        return outs[0], outs[1]

    def forces(self, model):
        outs, ptrs, kind = self._outputs([((self.n_atoms, 3), np.float64)])
        self._check(self._lib.mag_forces(self._h, C.byref(model), ptrs[0], kind))
        return outs[0]

    def forces_exact(self, model):
        """-dOmega/dR of the truncated-Krylov grand potential at the last
        solve's mu, differentiated through every column's Krylov space (see
        mag_forces_exact)."""
        outs, ptrs, kind = self._outputs([((self.n_atoms, 3), np.float64)])
        self._check(self._lib.mag_forces_exact(self._h, C.byref(model), ptrs[0], kind))
        return outs[0]

    def icohp(self, model):
        """(B, B_sigma, B_pi) per 4x4 block of the pattern, in block-CSR order
        (Eqs. 4-8; see mag_icohp)."""
        nblk = self.nnz // 16
        outs, ptrs, kind = self._outputs([((nblk,), np.float64)] * 3)
        self._check(self._lib.mag_icohp(self._h, C.byref(model), ptrs[0], ptrs[1], ptrs[2], kind))
        return outs

    def cohp(self, energies, eta):
        """C[block, q]: the COHP of each block of the pattern at energies[q] + i eta
        (Eq. 4; see mag_cohp).  Needs a solve with workflow="store"."""
        e = np.ascontiguousarray(np.asarray(energies, dtype=np.float64).ravel())
        nblk = self.nnz // 16
        outs, ptrs, kind = self._outputs([((nblk, e.size), np.float64)])
        self._check(self._lib.mag_cohp(self._h, e.ctypes.data_as(C.POINTER(C.c_double)), e.size,
                                       float(eta), ptrs[0], kind))
        return outs[0]

    # -------------------------------------------------------------- MD step
    def pair_repulsion(self, phi0, m_rep):
        """(E_rep, e_atom, F_rep) of the pair term on the last sk_build
        (see mag_pair_repulsion)."""
        outs, ptrs, kind = self._outputs([((self.sk_n,), np.float64), ((self.sk_n, 3), np.float64)])
        e = C.c_double()
        self._check(self._lib.mag_pair_repulsion(self._h, float(phi0), float(m_rep), C.byref(e),
                                                 ptrs[0], ptrs[1], kind))
        return e.value, outs[0], outs[1]

    def md_run(self, model, pos, vel, cell, dt, mass, n_steps, phi0=0.0, m_rep=4.0,
               r_cluster=0.0, exact_forces=False, **kw):
        """n_steps of velocity Verlet (see mag_md_run).  Returns (pos, vel, F,
        thermo) at the end; thermo[k] = (E_pot, E_kin, mu, E_band, E_rep) of
        frame k (frame 0: the start)."""
        o = make_opts(**kw)
        md = L.MagMDOpts(dt=float(dt), mass=float(mass), phi0=float(phi0), m_rep=float(m_rep),
                         r_cluster=float(r_cluster), n_steps=int(n_steps),
                         exact_forces=int(bool(exact_forces)))
        n = int(pos.shape[0])
        outs, ptrs, kind = self._outputs([((n, 3), np.float64)] * 3)
        for dst, src in zip(outs[:2], (pos, vel)):
            if self.device_outputs:
                dst.copy_(src if _is_dev(src) else torch.as_tensor(np.asarray(src, np.float64)))
            else:
                np.copyto(dst, src.detach().cpu().numpy() if _is_dev(src) else np.asarray(src))
        cellv = (C.c_double * 3)(*[float(x) for x in cell])
        thermo = np.zeros((int(n_steps) + 1, 5), dtype=np.float64)
        self._check(self._lib.mag_md_run(self._h, C.byref(model), C.byref(o), C.byref(md), n, cellv,
                                         ptrs[0], ptrs[1], ptrs[2],
                                         thermo.ctypes.data_as(C.POINTER(C.c_double)), kind))
        # the context now holds the last frame's build, system and solve
        rowptr = np.empty(4 * n + 1, dtype=np.int64)
        self._check(self._lib.mag_sk_get_csr(self._h, C.c_void_p(rowptr.ctypes.data), None, None,
                                             None, L.MAG_HOST))
        self.sk_n = self.n_atoms = n
        self.sk_nnz = self.nnz = int(rowptr[-1])
        self.opts = o
        return outs[0], outs[1], outs[2], thermo

    def stats(self):
        s = L.MagStats()
        self._check(self._lib.mag_get_stats(self._h, C.byref(s)))
        out = {}
        for name, _ in L.MagStats._fields_:
            v = getattr(s, name)
            out[name] = list(v) if isinstance(v, C.Array) else v
        return out


__all__ = ["Context", "MagError", "make_opts"]
