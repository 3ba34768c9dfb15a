"""C-ABI checks that need no GPU: the library loads, exports every declared symbol, and
descriptor validation rejects bad plans before any device work."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    from paper_2505_22718_amd import binding
    return binding.load()


def _declared_functions():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            text = open(os.path.join(ROOT, "include", fn)).read()
            names |= set(re.findall(r"^\s*(?:swiftcl_status|const char\*)\s+(swiftcl_\w+)\s*\(", text, re.M))
    return names


def test_exports_every_declared_symbol(lib):
    names = _declared_functions()
    assert {"swiftcl_plan", "swiftcl_windows", "swiftcl_cl", "swiftcl_cl_backward"} <= names
    for n in names:
        assert hasattr(lib, n), n


def _desc(**over):
    from paper_2505_22718_amd import binding as bd
    import synth
    k = np.geomspace(1e-4, 10, 256)
    ell = np.geomspace(2, 200, 20)
    zg = np.linspace(0.01, 3, 1024)
    zs = np.linspace(0.01, 3, 200)
    arrays = dict(k=k, ell=ell, z_geom=zg, z_nz=zs)
    arrays.update({a: over.pop(a) for a in list(over) if a in arrays})
    keep = {a: np.ascontiguousarray(v, dtype=np.float64) for a, v in arrays.items()}
    d = bd.swiftcl_plan_desc()
    d.n_chi = 512
    d.n_bands = 3
    for j, v in enumerate((0.0, 3.0, 6.0)):
        d.band_ell_lo[j] = v
    for kind, row in enumerate(((0.1, -0.2, -0.5), (-1.5, -2.0, -2.5), (-1.0, -1.0, -2.0))):
        for j, v in enumerate(row):
            d.fftlog_b[kind][j] = v
    dp = ctypes.POINTER(ctypes.c_double)
    d.n_k, d.k = len(keep["k"]), keep["k"].ctypes.data_as(dp)
    d.n_ell, d.ell = len(keep["ell"]), keep["ell"].ctypes.data_as(dp)
    d.n_zg, d.z_geom = len(keep["z_geom"]), keep["z_geom"].ctypes.data_as(dp)
    d.n_zs, d.z_nz = len(keep["z_nz"]), keep["z_nz"].ctypes.data_as(dp)
    d.max_batch, d.max_tracers, d.max_ell, d.precision, d.device = 1, 2, 20, 0, 0
    for key, v in over.items():
        if key.startswith("fftlog_b"):  # fftlog_b<kind><band>
            d.fftlog_b[int(key[-2])][int(key[-1])] = v
        else:
            setattr(d, key, v)
    return d, keep


@pytest.mark.parametrize("over,code", [
    (dict(n_chi=500), -1),                                   # not a power of two
    (dict(n_chi=8192), -5),                                  # a power of two that is not built
    (dict(n_chi=4096, n_k=256), -5),                         # 4096 not built
    (dict(k=np.linspace(1e-4, 10, 256)), -2),                # k not log-spaced
    (dict(k=np.geomspace(1e-4, 10, 1024)), -1),              # n_k > n_chi
    (dict(ell=np.geomspace(1.5, 200, 20)), -2),              # l < 2
    (dict(ell=np.array([2.0, 5.0, 4.0])), -1),               # not increasing
    (dict(fftlog_b00=1.2), -2),                              # b >= 1 outside eq. int_jl range
    (dict(fftlog_b20=1.0), -2),                              # the CMB-lensing row is checked too
    (dict(fftlog_b12=-7.8), -2),                             # b <= -l-1 at l = 6.72 (band 2)
    # RSD needs U at l - 2, magnification U at b - 2: the clustering b must exceed 1 - l
    (dict(precision=1, rsd=1, fftlog_b00=-1.5), -2),         # l = 2: b = -1.5 <= -1
    (dict(precision=1, magnification=1, fftlog_b01=-2.5), -2),  # l = 3.1: b = -2.5 <= -2.1
    (dict(n_bands=0), -1),
    (dict(taper_frac=1.0), -1),
    (dict(max_tracers=33), -5),
    (dict(max_batch=0), -1),
    (dict(precision=7), -1),
    (dict(edge_node=600), -1),
    (dict(z_nz=np.linspace(0.0, 3, 200)), -1),               # n(z) grid outside the geometry range
    (dict(k=np.array([1e-4] + [np.nan] * 255)), -1),
    (dict(n_interp=1), -1),                                  # one node cannot be interpolated
    (dict(n_interp=257), -1),                                # more nodes than k nodes
    (dict(n_interp=16), -5),                                 # scale-dependent growth in FP64
    (dict(rsd=1), -5),                                       # RSD in FP64
    (dict(rsd=2), -1),
    (dict(magnification=1), -5),                             # magnification in FP64
])
def test_plan_rejects_bad_descriptor(lib, over, code):
    d, keep = _desc(**over)
    h = ctypes.c_void_p()
    st = lib.swiftcl_plan(ctypes.byref(d), None, ctypes.byref(h))
    assert st == code, lib.swiftcl_last_error()
    assert h.value is None
    assert len(lib.swiftcl_last_error()) > 0


def test_null_arguments_rejected(lib):
    from paper_2505_22718_amd import binding as bd
    h = ctypes.c_void_p()
    assert lib.swiftcl_plan(None, None, ctypes.byref(h)) == bd.SWIFTCL_E_INVALID
    d, keep = _desc()
    assert lib.swiftcl_plan(ctypes.byref(d), None, None) == bd.SWIFTCL_E_INVALID
    inp = bd.swiftcl_inputs()
    assert lib.swiftcl_cl(None, ctypes.byref(inp), None, None) == bd.SWIFTCL_E_INVALID
    assert lib.swiftcl_windows(None, ctypes.byref(inp), None, None) == bd.SWIFTCL_E_INVALID
    assert lib.swiftcl_cl_backward(None, ctypes.byref(inp), None, None, None, None, None, 0, None) == bd.SWIFTCL_E_INVALID
    assert lib.swiftcl_cl_backward(None, ctypes.byref(inp), None, None, None, None, None,
                                   bd.SWIFTCL_BWD_REUSE_FORWARD, None) == bd.SWIFTCL_E_INVALID
    assert lib.swiftcl_cl_kgrowth(None, ctypes.byref(inp), None, None, None) == bd.SWIFTCL_E_INVALID
    assert lib.swiftcl_cl_limber(None, ctypes.byref(inp), None, None) == bd.SWIFTCL_E_INVALID
    assert lib.swiftcl_plan_destroy(None) == bd.SWIFTCL_E_INVALID


def _header_fields(struct):
    """Field names of a typedef'd struct in include/swiftcl.h, in order (array fields by name)."""
    text = open(os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                             "include", "swiftcl.h")).read()
    text = re.sub(r"//[^\n]*", "", re.sub(r"/\*.*?\*/", "", text, flags=re.S))
    body = re.search(r"typedef struct \{([^{}]*)\}\s*" + struct + r"\s*;", text).group(1)
    names = []
    for decl in body.split(";"):
        decl = decl.strip()
        if decl:
            names.append(re.match(r".*?(\w+)\s*(\[[^\]]*\])*\s*$", decl, flags=re.S).group(1))
    return names


@pytest.mark.parametrize("struct", ["swiftcl_plan_desc", "swiftcl_inputs"])
def test_binding_structs_match_the_header(struct):
    from paper_2505_22718_amd import binding as bd
    got = [name for name, _ in getattr(bd, struct)._fields_]
    assert got == _header_fields(struct)


@pytest.mark.parametrize("struct", ["swiftcl_plan_desc", "swiftcl_inputs"])
def test_binding_struct_offsets_match_a_c_compiler(struct, tmp_path):
    """sizeof and every field's offsetof as gcc lays the header's struct out, against ctypes."""
    import shutil
    import subprocess
    from paper_2505_22718_amd import binding as bd
    if shutil.which("gcc") is None:
        pytest.skip("no gcc")
    cls = getattr(bd, struct)
    inc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")
    lines = ['#include "swiftcl.h"', "#include <stdio.h>", "#include <stddef.h>", "int main(void) {",
             f'  printf("%zu\\n", sizeof({struct}));']
    lines += [f'  printf("%zu\\n", offsetof({struct}, {name}));' for name, _ in cls._fields_]
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-Wall", "-Werror", "-I", inc, str(src), "-o", str(exe)], check=True)
    got = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()]
    want = [ctypes.sizeof(cls)] + [getattr(cls, name).offset for name, _ in cls._fields_]
    assert got == want


def _header_prototypes():
    """{name: [parameter declarations]} of every function include/swiftcl.h declares."""
    text = open(os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                             "include", "swiftcl.h")).read()
    text = re.sub(r"//[^\n]*", "", re.sub(r"/\*.*?\*/", "", text, flags=re.S))
    protos = {}
    for m in re.finditer(r"(?:swiftcl_status|const\s+char\s*\*)\s*(swiftcl_\w+)\s*\(([^)]*)\)\s*;", text):
        body = " ".join(m.group(2).split())
        protos[m.group(1)] = [] if body == "void" else [p.strip() for p in body.split(",")]
    return protos


def test_binding_argtypes_match_the_header(lib):
    """Every prototype's parameter count, and for each parameter pointer versus 32-bit integer (signed
    or not), against the ctypes argtypes the binding declares; status returns are int, the error
    message a C string."""
    from paper_2505_22718_amd import binding as bd
    protos = _header_prototypes()
    assert set(protos) == set(bd.EXPORTED)
    for name, params in protos.items():
        f = getattr(lib, name)
        argtypes = list(f.argtypes or [])
        assert len(argtypes) == len(params), name
        for p, a in zip(params, argtypes):
            pointer = "*" in p or p.startswith("swiftcl_plan_t")
            if pointer:
                assert a in (ctypes.c_void_p, ctypes.c_char_p) or issubclass(a, ctypes._Pointer), (name, p)
            else:
                want = ctypes.c_uint32 if p.startswith("uint32_t") else ctypes.c_int32
                assert a is want, (name, p)
        assert f.restype is (ctypes.c_char_p if name == "swiftcl_last_error" else ctypes.c_int), name
