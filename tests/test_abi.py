"""The C-ABI library loads and exports every function include/lbm.h declares; host-side
validation works without a GPU (no compute is launched here)."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "lbm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*((?:lbm|ib)_[a-z_0-9]+)\s*\(", src, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_boundary_calls():
    names = declared_functions()
    for must in ["lbm_create", "lbm_step", "ib_spread", "ib_interp", "lbm_moments"]:
        assert must in names
    assert len(names) >= 20


def test_library_exports_every_declared_symbol():
    from paper_1312_2234_amd import lbm

    L = lbm.lib()
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert not missing, missing
    assert set(declared_functions()) <= set(lbm.EXPORTS)


def _params(**kw):
    from paper_1312_2234_amd import lbm

    d = dict(nx=32, ny=32, nz=32, walls=1, tau=0.8)
    d.update(kw)
    p = lbm.LbmParams(d["nx"], d["ny"], d["nz"], d["walls"], d["tau"], (C.c_float * 3)(0, 0, 0),
                      (C.c_float * 3)(0, 0, 0), (C.c_float * 3)(*(d.get("uhi", (0, 0, 0)))))
    return (lbm.LbmParams * 1)(p)


def test_workspace_size_and_validation():
    from paper_1312_2234_amd import lbm

    L = lbm.lib()
    ok = L.lbm_workspace_bytes(_params(), 1, 0, 0)
    assert ok >= 2 * 19 * 32 ** 3 * 4
    half = L.lbm_workspace_bytes(_params(), 1, 1, 0)
    assert half < ok and half >= 2 * 19 * 32 ** 3 * 2
    assert L.lbm_workspace_bytes(_params(tau=0.5), 1, 0, 0) == 0          # tau must exceed 1/2
    assert L.lbm_workspace_bytes(_params(nx=0), 1, 0, 0) == 0
    assert L.lbm_workspace_bytes(_params(uhi=(0, 0.1, 0)), 1, 0, 0) == 0  # wall-normal wall speed
    assert L.lbm_workspace_bytes(_params(), 1, 7, 0) == 0                 # unknown storage
    assert L.lbm_workspace_bytes(_params(), 1, 0, 1000) > ok              # IB buffers


def test_create_rejects_bad_arguments_on_host():
    from paper_1312_2234_amd import lbm

    L = lbm.lib()
    h = C.c_void_p()
    assert L.lbm_create(_params(), 1, 0, 0, 0, None, 0, None, C.byref(h)) == 1       # no workspace
    assert L.lbm_create(_params(tau=0.4), 1, 0, 0, 0, C.c_void_p(256), 1 << 30, None, C.byref(h)) == 1
    assert L.lbm_create(_params(), 1, 0, 0, 0, C.c_void_p(256), 16, None, C.byref(h)) == 1  # too small
    assert L.lbm_create(_params(), 1, 0, 0, 0, C.c_void_p(257), 1 << 30, None, C.byref(h)) == 1  # misaligned
    assert L.lbm_create(_params(nx=3), 1, 0, 0, 10, C.c_void_p(256), 1 << 30, None, C.byref(h)) == 4  # IB needs nx>=4
    assert h.value is None
    assert L.lbm_step(None, 1) == 1 and L.ib_spread(None, 0, None, None) == 1
    assert L.lbm_status_string(3) == b"HIP error"


def test_oracle_builds_and_is_separate():
    """The oracle is its own gcc-built library; the GPU sources never include it."""
    from oracle import oracle

    assert os.path.exists(oracle.build(force=False))
    csrc = os.path.join(ROOT, "paper_1312_2234_amd", "csrc")
    for f in os.listdir(csrc):
        assert "oracle" not in open(os.path.join(csrc, f)).read()


def test_bench_refuses_more_than_one_gpu():
    """The benchmark measures one GPU; asked for more it says so and exits non-zero, before
    touching a device."""
    import os
    import subprocess
    import sys

    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=root)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)


def test_ctypes_structs_match_the_c_layout(tmp_path):
    """The binding's ctypes mirrors of lbm_params, lbm_launch and ib_membrane have the C
    header's field offsets and sizes (a C program built against include/lbm.h prints them)."""
    import subprocess

    from paper_1312_2234_amd import lbm

    structs = {"lbm_params": lbm.LbmParams, "lbm_launch": lbm.LbmLaunch, "ib_membrane": lbm.IbMembrane}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "lbm.h"', "int main(void) {"]
    for cname, cls in structs.items():
        lines.append('    printf("%s %%zu\\n", sizeof(%s));' % (cname, cname))
        for f, _ in cls._fields_:
            lines.append('    printf("%s.%s %%zu\\n", offsetof(%s, %s));' % (cname, f, cname, f))
    lines += ["    return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = dict(l.split() for l in subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.splitlines())
    for cname, cls in structs.items():
        assert int(got[cname]) == C.sizeof(cls), cname
        for f, _ in cls._fields_:
            assert int(got["%s.%s" % (cname, f)]) == getattr(cls, f).offset, (cname, f)


def test_wall_kinds_validated_on_host():
    from paper_1312_2234_amd import lbm

    L = lbm.lib()
    assert L.lbm_workspace_bytes(_params(walls=2), 1, 0, 0) > 0          # on-site walls
    assert L.lbm_workspace_bytes(_params(walls=3), 1, 0, 0) == 0         # unknown wall kind
    assert L.lbm_workspace_bytes(_params(walls=2, ny=2), 1, 0, 0) == 0   # two wall rows, no fluid row
    assert L.lbm_workspace_bytes(_params(walls=1, ny=2), 1, 0, 0) > 0


def test_bench_workloads_build():
    """Every workload bench.py names builds on the host with the shape its description states."""
    import importlib.util

    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    bench = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(bench)
    chans, desc = bench.make_workload("shear")
    assert (chans[0].nx, chans[0].ny, chans[0].nz) == (256, 128, 128) and chans[0].bodies.n == 16 * 2562
    assert chans[0].walls is True and chans[0].bodies.triangles is None
    chans, desc = bench.make_workload("shear_large")
    assert (chans[0].nx, chans[0].ny, chans[0].nz) == (512, 256, 128) and chans[0].bodies.n == 64 * 2562
    chans, desc = bench.make_workload("shear_onsite")
    assert chans[0].walls == "onsite" and "on-site" in desc
    chans, desc = bench.make_workload("shear_constrained")
    b = chans[0].bodies
    assert b.triangles is not None and len(b.triangles) == 16 * 5120 and b.k_volume > b.k_area_global > 0
    chans, desc = bench.make_workload("shear_fe")
    b = chans[0].bodies
    assert b.elements6 is not None and b.elements6.shape == (16 * 1280, 6) and b.k_bend == 0.0
    assert abs(b.k_fe / 2.53e-4 - 1) < 1e-2 and "Eq. 6-10" in desc
    chans, desc = bench.make_workload("shear_adhesion")
    a = bench.adhesion_of("shear_adhesion", chans)
    assert len(a["rec_tri"]) == 16 * 5344 and len(a["ligands"]) == 256 * 128 and abs(a["capture"] - 0.64) < 1e-12
    assert chans[0].bodies.X[1].min() > -0.5 and chans[0].bodies.X[1].min() < -0.5 + a["capture"]
    assert bench.adhesion_of("shear", chans) is None
    chans, desc = bench.make_workload("batched")
    assert len(chans) == 64
    chans, desc = bench.make_workload("coarse")
    assert (chans[0].nx, chans[0].ny, chans[0].nz) == (128, 64, 64)
    with pytest.raises(SystemExit):
        bench.make_workload("nonexistent")
