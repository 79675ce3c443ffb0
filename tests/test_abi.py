"""The C ABI without a GPU: the library loads, exports every entry point of
include/mag.h, and the ctypes structures match the C layout."""
import ctypes as C
import os
import re
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mag.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mag_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = _declared()
    for n in ["mag_create", "mag_set_system", "mag_solve_columns", "mag_density_matrix",
              "mag_energy", "mag_backward", "mag_forces", "mag_green_columns", "mag_sk_build"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_1210_1531_amd import _lib as L
    lib = L.load()
    names = _declared()
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    assert set(names) == set(L.PROTOTYPES), set(names) ^ set(L.PROTOTYPES)
    out = subprocess.run(["nm", "-D", "--defined-only", L.LIB_PATH], capture_output=True,
                         text=True).stdout
    exported = set(re.findall(r"\bT (mag_\w+)", out))
    assert set(names) <= exported


def test_struct_layouts_match_c():
    from paper_1210_1531_amd import _lib as L
    src = r"""
#include <stdio.h>
#include <stddef.h>
#include "mag.h"
#define P(T, f) printf(#T "." #f " %zu\n", offsetof(T, f))
int main(void) {
  printf("mag_sk_model %zu\n", sizeof(mag_sk_model));
  printf("mag_system %zu\n", sizeof(mag_system));
  printf("mag_opts %zu\n", sizeof(mag_opts));
  printf("mag_stats %zu\n", sizeof(mag_stats));
  P(mag_system, cell); P(mag_system, r_cluster); P(mag_system, clus_atoms);
  P(mag_opts, mu_fixed); P(mag_opts, workflow); P(mag_opts, schedule);
  P(mag_stats, n_columns); P(mag_stats, bisect_levels); P(mag_stats, schedule_used);
  P(mag_stats, t_krylov_ms); P(mag_stats, krylov_launches);
  P(mag_sk_model, r_cut);
  return 0;
}
"""
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "layout.c")
        exe = os.path.join(d, "layout")
        open(c, "w").write(src)
        subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), c, "-o", exe],
                       check=True)
        out = subprocess.run([exe], capture_output=True, text=True, check=True).stdout
    got = dict(line.rsplit(" ", 1) for line in out.strip().splitlines())
    types = {"mag_sk_model": L.MagSKModel, "mag_system": L.MagSystem, "mag_opts": L.MagOpts,
             "mag_stats": L.MagStats}
    for k, v in got.items():
        v = int(v)
        if "." in k:
            t, f = k.split(".")
            assert getattr(types[t], f).offset == v, k
        else:
            assert C.sizeof(types[k]) == v, k


def test_host_only_entry_points():
    from paper_1210_1531_amd import _lib as L, make_opts
    lib = L.load()
    assert lib.mag_version() >= 100
    assert lib.mag_last_error(None) == b"context is NULL"
    o = make_opts(nu=20, kT=0.2, n_electrons=8.0)
    assert o.nu == 20 and o.kT == 0.2 and o.mu_fixed != o.mu_fixed  # NaN
    assert o.workflow == L.MAG_WORKFLOW_AUTO and o.schedule == L.MAG_SCHED_AUTO
    assert lib.mag_create(None, 0, None) == L.MAG_EINVAL


def test_product_path_has_no_oracle_dependency():
    pkg = os.path.join(ROOT, "paper_1210_1531_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert "oracle" not in re.sub(r"#.*|//.*", "", text).lower() or f == "__init__.py", f


def test_missing_library_fails_loudly(monkeypatch):
    from paper_1210_1531_amd import _lib as L
    monkeypatch.setattr(L, "_lib", None)
    monkeypatch.setattr(L, "LIB_PATH", "/nonexistent/libmag.so")
    with pytest.raises(RuntimeError, match="not built"):
        L.load()
