"""CPU checks of the C-ABI boundary: the library loads, exports every symbol
the header declares, the descriptor layout seen by the binding matches the
C compiler's, and argument validation works without touching a GPU."""
import ctypes as C
import os
import re
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sgpm.h")


def _lib():
    import paper_2404_19602_amd._lib as L
    if not os.path.exists(L.LIB_PATH):
        from paper_2404_19602_amd import build
        build.build()
    return L


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sgpm_[a-z_0-9]+)\s*\(", text)))


def test_every_declared_symbol_is_exported():
    L = _lib()
    lib = C.CDLL(L.LIB_PATH)
    names = declared_functions()
    assert len(names) >= 20
    for n in names:
        assert hasattr(lib, n), n
    out = subprocess.run(["nm", "-D", "--defined-only", L.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r" T (sgpm_[a-z_0-9]+)", out))
    assert set(names) <= exported
    # nothing else with the prefix leaks out undeclared
    assert exported <= set(names)


def test_descriptor_layout_matches_c():
    L = _lib()
    fields = [f[0] for f in L.Desc._fields_]
    src = ['#include <stdio.h>', '#include <stddef.h>', f'#include "{HEADER}"', "int main(void){",
           'printf("%zu\\n", sizeof(sgpm_instance_desc));']
    for f in fields:
        cf = "instance_id" if f == "instance_id" else f
        src.append(f'printf("%zu\\n", offsetof(sgpm_instance_desc, {cf}));')
    src.append("return 0;}")
    with tempfile.TemporaryDirectory() as d:
        cpath = os.path.join(d, "probe.c")
        open(cpath, "w").write("\n".join(src))
        exe = os.path.join(d, "probe")
        subprocess.run(["gcc", "-std=c11", "-o", exe, cpath], check=True)
        vals = [int(x) for x in subprocess.run([exe], capture_output=True, text=True,
                                               check=True).stdout.split()]
    assert vals[0] == C.sizeof(L.Desc)
    for f, off in zip(fields, vals[1:]):
        assert getattr(L.Desc, f).offset == off, f


def test_default_descriptor_is_the_papers():
    L = _lib()
    lib = L.lib()
    d = L.Desc()
    lib.sgpm_default_desc(C.byref(d))
    assert d.nk == 240 and d.lk_eV == 5.0 and d.alpha == 0.1
    assert d.fermi_eV == 0.4 and d.temp_K == 300.0 and d.pauli == 1
    assert list(d.rate_scale) == [1.0] * 6


def _desc(**kw):
    L = _lib()
    d = L.Desc()
    L.lib().sgpm_default_desc(C.byref(d))
    for k, v in kw.items():
        setattr(d, k, v)
    return d


def test_workspace_bytes_and_validation():
    L = _lib()
    lib = L.lib()
    nb = C.c_size_t(0)
    d = _desc(dim_z=1, degree=5, nodes_1d=8, gap_dim=0, gap_rel=0.1, n_particles=1000)
    assert lib.sgpm_workspace_bytes(C.byref(d), 1, C.byref(nb)) == 0
    state = 2 * 6 * 1000 * 8
    hist = 3 * 8 * 240 * 240 * 4
    assert nb.value >= state + hist
    d32 = _desc(dim_z=1, degree=5, nodes_1d=8, gap_dim=0, gap_rel=0.1, n_particles=1000, precision=1)
    nb32 = C.c_size_t(0)
    assert lib.sgpm_workspace_bytes(C.byref(d32), 1, C.byref(nb32)) == 0
    assert nb.value - nb32.value >= state // 2 - 4096
    bad = [dict(n_particles=0), dict(dim_z=3), dict(temp_K=-1.0), dict(nk=1), dict(c_max=0),
           dict(c_max=300), dict(dim_z=1, gap_dim=1), dict(gap0=-0.1), dict(precision=7),
           dict(dim_z=1, degree=40, nodes_1d=41, gap_dim=0), dict(max_steps=-1),
           dict(pauli=2), dict(alpha=-0.5),
           # Q nk^2 = 121 * 4096^2 > 2^30: cell offsets would leave 32 bits
           dict(dim_z=2, degree=2, nodes_1d=11, gap_dim=0, nk=4096)]
    for b in bad:
        db = _desc(**b)
        assert lib.sgpm_workspace_bytes(C.byref(db), 1, C.byref(nb)) == 1, b
    # the largest grid with 8 nodes stays within the 32-bit cell offsets
    dbig = _desc(dim_z=1, degree=5, nodes_1d=8, gap_dim=0, nk=4096)
    assert lib.sgpm_workspace_bytes(C.byref(dbig), 1, C.byref(nb)) == 0
    assert lib.sgpm_workspace_bytes(None, 1, C.byref(nb)) == 1
    assert lib.sgpm_workspace_bytes(C.byref(d), 0, C.byref(nb)) == 1


def test_create_rejects_missing_workspace_without_device_work():
    L = _lib()
    lib = L.lib()
    d = _desc(n_particles=100)
    ctx = C.c_void_p(0)
    assert lib.sgpm_create(C.byref(d), 1, None, 0, None, C.byref(ctx)) == 3   # EWORKSPACE
    assert not ctx.value
    assert lib.sgpm_create(C.byref(d), 1, C.c_void_p(256), 10, None, C.byref(ctx)) == 3
    dbad = _desc(n_particles=0)
    assert lib.sgpm_create(C.byref(dbad), 1, C.c_void_p(256), 1 << 40, None, C.byref(ctx)) == 1
    assert lib.sgpm_status_string(4) == b"device error"


def test_null_context_calls_fail_cleanly():
    lib = _lib().lib()
    assert lib.sgpm_step(None, 1e-15, 1) == 1
    assert lib.sgpm_init_particles(None) == 1
    n = C.c_int64(0)
    assert lib.sgpm_record_length(None, 0, C.byref(n)) == 1
    assert lib.sgpm_last_error(None) == b"null context"
    lib.sgpm_destroy(None)


def test_product_never_imports_the_oracle():
    pkg = os.path.join(ROOT, "paper_2404_19602_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".cpp", ".hip", ".h")):
                text = open(os.path.join(dirpath, f)).read()
                assert "oracle" not in text.lower().replace("the oracle", ""), f


def test_noalloc_validation_without_device_work():
    """sgpm_energy_density_noalloc refuses bad arguments before touching a
    device: null pointers, a bad precision, and more bins than its fixed
    scratch holds (Q * nbins > 2^19)."""
    L = _lib()
    lib = L.lib()
    f = lib.sgpm_energy_density_noalloc
    one = C.c_void_p(1)
    args = lambda **kw: dict(dict(kx=one, ky=one, prec=0, n=C.c_int64(10), P=6, Q=8, psi=one,
                                  eps0=one, nbins=256, emin=C.c_double(0.0),
                                  emax=C.c_double(2.0), out=one, stream=None), **kw)
    call = lambda a: f(a["kx"], a["ky"], a["prec"], a["n"], a["P"], a["Q"], a["psi"], a["eps0"],
                       a["nbins"], a["emin"], a["emax"], a["out"], a["stream"])
    assert call(args(kx=None)) == 1
    assert call(args(out=None)) == 1
    assert call(args(prec=3)) == 1
    assert call(args(emax=C.c_double(0.0))) == 1
    assert call(args(Q=128, nbins=4097)) == 6
