"""The C ABI: the library loads and exports every entry point of include/tribo.h,
and rejects invalid configurations on the host (no GPU needed)."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2602_10761_amd import runtime as R

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "tribo.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(tf_[a-z_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("tf_init", "tf_step", "tf_adjoint_step", "tf_stats", "tf_workspace_size", "tf_get_state",
              "tf_set_state", "tf_set_params", "tf_poisson", "tf_field", "tf_destroy", "tf_error_string",
              "tf_last_error"):
        assert n in names


def test_library_exports_every_declared_symbol():
    L = R.lib()
    for n in declared_functions():
        assert hasattr(L, n), n


def cfg(nx=32, ny=16, nz=32, n=100, **kw):
    yf = np.linspace(0.0, 360.0, ny + 1)
    c = R.TfEnsemble()
    c.nx, c.ny, c.nz, c.n_particles = nx, ny, nz, n
    c.lx, c.lz = 100.0, 50.0
    c.y_faces = yf.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    c.dt, c.density_ratio, c.k_c, c.delta_u, c.e, c.c_el = 0.1, 1000.0, 1e-3, 1.0, 0.9, 1.0
    c.un_bin = 0.05
    c.u_nodes = 4096
    for k, v in kw.items():
        setattr(c, k, v)
    return c, yf


def ws(c):
    arr = (R.TfEnsemble * 1)(c)
    return R.lib().tf_workspace_size(arr, 1, 0)


def test_workspace_size_valid_and_monotone():
    c, yf = cfg()
    a = ws(c)
    c2, yf2 = cfg(n=10000)
    assert 0 < a < ws(c2)


@pytest.mark.parametrize("bad", [dict(nx=7), dict(nx=14), dict(nz=2), dict(nx=512), dict(ny=1),
                                 dict(n_particles=-1), dict(dt=0.0), dict(e=0.0), dict(e=1.5),
                                 dict(density_ratio=-1.0), dict(u_nodes=None), dict(un_bin=0.0)])
def test_invalid_configs_rejected(bad):
    c, yf = cfg(**bad)
    assert ws(c) == 0


def test_non_monotone_faces_rejected():
    c, yf = cfg()
    yf[3] = yf[2]
    assert ws(c) == 0
    c, yf = cfg()
    yf[0] = 1.0
    assert ws(c) == 0


def test_init_rejects_without_touching_device():
    L = R.lib()
    c, yf = cfg(nx=9)
    h = ctypes.c_void_p()
    rc = L.tf_init((R.TfEnsemble * 1)(c), 1, (R.TfParticles * 1)(), ctypes.c_void_p(256), 1 << 20, 0, None, 0,
                   ctypes.byref(h))
    assert rc == -1 and not h.value
    assert b"nx" in L.tf_last_error()
    assert L.tf_error_string(-2) == b"size limit or workspace too small"


def test_bench_traffic_file_parsing(tmp_path, monkeypatch):
    # the committed HBM traffic summary carries comments after the values
    import bench
    f = tmp_path / "traffic.txt"
    f.write_text("# header\nsource_hash: abc\npush_bytes: 123   # fetch 1 KiB raw\nsort_bytes: 7\n")
    monkeypatch.setattr(bench, "traffic_file", lambda config: str(f))
    monkeypatch.setattr(bench, "source_hash", lambda: "abc")
    assert bench.measured_traffic("push", 3) == 123.0
    assert bench.measured_traffic("sort", 3) == 7.0
    assert bench.measured_traffic("tridiag", 3) is None
    monkeypatch.setattr(bench, "source_hash", lambda: "other")
    assert bench.measured_traffic("push", 3) is None


def test_bench_byte_accounting():
    # the method's own bytes per step at the 4e6-particle 192x160x192 workload
    # (N_p < N_c): 120 N_p + 24 N_c (carrier) + 8 N_p (deposit) + 16 N_c
    # (Poisson) + 8 N_c (stencil) = 795.1 MB
    import bench
    n_p, nx, ny, nz = 4_000_000, 192, 160, 192
    n_c = nx * ny * nz
    assert bench.algorithmic_step_bytes(n_p, nx, ny, nz) == 128 * n_p + 48 * n_c
    assert abs(bench.algorithmic_step_bytes(n_p, nx, ny, nz) / 1e6 - 795.1) < 0.05
    assert bench.algorithmic_push_bytes(n_p, nx, ny, nz) == 120 * n_p + 32 * n_c
    # sparse particles: carrier and stencil by particle
    assert bench.algorithmic_push_bytes(10, 64, 64, 64) == 120 * 10 + 192 * 10 + 56 * 10
    # the design moves at least the method's bytes
    assert bench.design_bytes("push", n_p, nx, ny, nz) > bench.algorithmic_push_bytes(n_p, nx, ny, nz)


def test_struct_layouts_match_header(tmp_path):
    # the ctypes mirrors of the ABI structs have the C layout (sizes and offsets)
    import shutil
    import subprocess
    from paper_2602_10761_amd import runtime as R
    if shutil.which("gcc") is None:
        pytest.skip("no C compiler")
    structs = {"tf_ensemble": R.TfEnsemble, "tf_particles": R.TfParticles, "tf_stats_out": R.TfStatsOut,
               "tf_tuning": R.TfTuning}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "tribo.h"', "int main(void) {"]
    for name, cls in structs.items():
        lines.append(f'  printf("{name} %zu\\n", sizeof({name}));')
        for f in cls._fields_:
            lines.append(f'  printf("{name}.{f[0]} %zu\\n", offsetof({name}, {f[0]}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    inc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")
    subprocess.run(["gcc", "-I", inc, str(src), "-o", str(exe)], check=True)
    got = dict(l.split() for l in subprocess.run([str(exe)], check=True, capture_output=True,
                                                   text=True).stdout.splitlines())
    for name, cls in structs.items():
        assert int(got[name]) == ctypes.sizeof(cls), name
        for f in cls._fields_:
            assert int(got[f"{name}.{f[0]}"]) == getattr(cls, f[0]).offset, f"{name}.{f[0]}"


def test_autotune_candidates():
    # the layouts the tuner tries are the ones the library accepts (mirrored
    # limits), and the sort capacities bracket the mean row-pair population
    from paper_2602_10761_amd import autotune as A
    from paper_2602_10761_amd import workload as W
    assert A.inverse_layouts(192, 192) == [4, 3]
    assert A.inverse_layouts(128, 128) == [1, 2, 4, 3]
    assert A.inverse_layouts(8, 12) == [1, 2, 3]
    for n in (300_000, 2_000_000):
        ens = W.make_workload(3, n_particles=n)[0]
        mean = n / (160 * 192 // 2)
        caps = A.sort_cap_candidates(ens)
        assert min(caps) <= max(mean, 64) < max(caps) <= max(2.5 * mean + 64, 128)
    assert all(c % 8 == 0 for c in caps)


def test_tuning_ranges():
    # host-side validation of tf_tuning (no device work)
    L = R.lib()
    try:
        assert L.tf_set_tuning(ctypes.byref(R.TfTuning(0, 0, 0, 0, 2))) == 0
        assert L.tf_set_tuning(ctypes.byref(R.TfTuning(0, 0, 0, 0, 3))) != 0
        assert L.tf_set_tuning(ctypes.byref(R.TfTuning(0, 0, 0, 5, 0))) != 0
        assert L.tf_set_tuning_class(8, 8, 8, ctypes.byref(R.TfTuning(0, 0, 0, 0, -1))) != 0
        assert L.tf_set_tuning_class(8, 8, 8, ctypes.byref(R.TfTuning(0, 0, 0, 0, 1))) == 0
        assert L.tf_set_tuning_class(8, 8, 8, None) == 0
    finally:
        assert L.tf_set_tuning(None) == 0


def test_bench_source_hash_ignores_comments(tmp_path, monkeypatch):
    # a measurement stays valid across comment edits, not across code edits
    import bench
    src = tmp_path / "k.hip"
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "KERNEL_SOURCES", ["k.hip"])
    src.write_text("int f(int a) { return a + 1; }  // one\n/* block\n comment */\n")
    h0 = bench.source_hash()
    src.write_text("// new header\nint f(int a) { return a + 1; }  // two\n\n")
    assert bench.source_hash() == h0
    src.write_text("int f(int a) { return a + 2; }\n")
    assert bench.source_hash() != h0
