"""The library's host C++ under AddressSanitizer and UndefinedBehaviorSanitizer
(no GPU): a sanitized build of the host sources (linked with the regular
device objects) is driven, in a child process with the sanitizer runtime
preloaded, through every entry point that runs on the host alone -- cell
validation and planning (Miller lists, stick tables, box geometry) on valid
and malformed cells, projector-table validation, the Davidson / subspace /
density planning paths -- so that an out-of-bounds read, a use after free or
undefined arithmetic in them fails the test."""

import os
import subprocess
import sys
import textwrap

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = textwrap.dedent(r'''
    import ctypes, sys, os
    import numpy as np
    sys.path.insert(0, ROOT)
    import cellgen
    lib = ctypes.CDLL(LIB)
    # the binding's structures, bound to the sanitized library
    sys.modules.pop("paper_2104_10502_amd", None)
    import importlib.util
    spec = importlib.util.spec_from_file_location("qb", os.path.join(ROOT, "paper_2104_10502_amd", "__init__.py"))
    src = open(spec.origin).read()
    ns = {"_lib": lib}
    # only the ctypes structure definitions and the cell marshalling
    start = src.index("class QehProjgen")
    stop = src.index("def generate_beta")
    exec("import ctypes\nimport numpy as np\n_c_int_p = ctypes.POINTER(ctypes.c_int)\n"
         "_c_dbl_p = ctypes.POINTER(ctypes.c_double)\n_sz_p = ctypes.POINTER(ctypes.c_size_t)\n"
         + src[start:stop], ns)
    QehCell = ns["QehCell"]; cell_struct = ns["_cell_struct"]
    lib.qeh_ctx_plan.argtypes = [ctypes.POINTER(QehCell), ctypes.POINTER(ctypes.c_size_t)]
    lib.qeh_beta_plan.argtypes = [ctypes.POINTER(QehCell), ctypes.POINTER(ctypes.c_size_t)]
    lib.qeh_subspace_plan.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_size_t)]
    lib.qeh_last_error.restype = ctypes.c_char_p
    lib.qeh_status_str.restype = ctypes.c_char_p
    n = ctypes.c_size_t()
    seen = {}
    def plan(c, label, **kw):
        keep = []
        s = cell_struct(c.lattice, c.fft, c.kpt, c.miller, c.vloc, c.nproj, kw.get("beta", c.beta),
                        c.dmat, kw.get("prec", 0), kw.get("block", 16), keep,
                        projgen=kw.get("projgen"), gamma=kw.get("gamma", False),
                        qmat=kw.get("qmat"))
        st = lib.qeh_ctx_plan(ctypes.byref(s), ctypes.byref(n))
        seen[label] = st
        lib.qeh_last_error(); lib.qeh_status_str(st)
        if kw.get("projgen") is not None:
            lib.qeh_beta_plan(ctypes.byref(s), ctypes.byref(n))
        return st
    c1 = cellgen.make_cell("c1")
    assert plan(c1, "c1") == 0
    assert plan(c1, "c1 mixed", prec=1) == 0
    c1q = cellgen.make_cell("c1", overlap=True)
    assert plan(c1q, "c1 overlap", qmat=c1q.qmat) == 0
    h = cellgen.gamma_half(c1)
    assert plan(h, "c1 gamma", gamma=True) == 0
    sv = cellgen.random_served_cell(24, 25.0, 1, 3, with_beta=False)
    pg = cellgen.projgen_tables(sv)
    assert plan(sv, "served tables", beta=None, projgen=pg) == 0
    anis = cellgen.make_cell("c1", fft=(28, 30, 35))
    assert plan(anis, "radix-7 box") == 0
    # malformed cells: every one rejected with an error status
    import copy
    bad = copy.deepcopy(c1); bad.miller = bad.miller[::-1].copy()
    assert plan(bad, "unsorted miller") != 0
    bad = copy.deepcopy(c1); bad.miller = bad.miller.copy(); bad.miller[5] = (40, 0, 0)
    assert plan(bad, "miller outside box") != 0
    bad = copy.deepcopy(c1); bad.fft = (30, 30, 11)
    assert plan(bad, "prime 11 box") != 0
    bad = copy.deepcopy(c1); bad.miller = bad.miller[:1].copy(); bad.beta = bad.beta[:, :1].copy()
    assert plan(bad, "one plane wave") == 0
    bad = copy.deepcopy(h); bad.miller = bad.miller[1:].copy(); bad.beta = bad.beta[:, 1:].copy()
    assert plan(bad, "gamma without G=0", gamma=True) != 0
    pgb = dict(pg); pgb["tab"] = pg["tab"][:, :5].copy()
    assert plan(sv, "short table", beta=None, projgen=pgb) != 0
    assert plan(c1, "block 0", block=0) != 0
    for nn, nb in ((1, 1), (2048, 1024), (2049, 1), (4, 5), (0, 0)):
        lib.qeh_subspace_plan(nn, nb, ctypes.byref(n))
    print("ok", len(seen))
''')


@pytest.mark.slow
def test_host_code_under_asan_and_ubsan():
    sys.path.insert(0, os.path.join(ROOT, "paper_2104_10502_amd"))
    import importlib.util
    spec = importlib.util.spec_from_file_location(
        "qeh_build", os.path.join(ROOT, "paper_2104_10502_amd", "build.py"))
    b = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(b)
    lib = b.build_host_sanitized()
    rt = subprocess.run([os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "bin", "hipcc"),
                         "-print-file-name=libclang_rt.asan-x86_64.so"],
                        capture_output=True, text=True).stdout.strip()
    assert os.path.exists(rt), rt
    env = dict(os.environ, LD_PRELOAD=rt,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", HIP_VISIBLE_DEVICES="")
    code = "ROOT = %r\nLIB = %r\n" % (ROOT, lib) + CHILD
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=env,
                       timeout=600)
    print(r.stdout[-2000:], r.stderr[-4000:])
    assert r.returncode == 0, r.stderr[-4000:]
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr
    assert r.stdout.strip().startswith("ok")
