"""Host-side checks of the C-ABI library (no GPU needed): it loads, exports
every entry point include/pi.h declares, validates descriptors before touching
the device, and its host-only rate table matches the oracle's."""
import ctypes as C
import math
import os
import re

import numpy as np
import pytest

from paper_1201_5651_amd import binding, synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "pi.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return set(re.findall(r"\b(pi_[a-z0-9_]+)\s*\(", text))


def test_library_loads_and_exports_every_declared_symbol():
    L = binding.lib()
    decl = declared_symbols()
    assert decl == set(binding.ABI_SYMBOLS), decl ^ set(binding.ABI_SYMBOLS)
    for name in decl:
        assert hasattr(L, name), name
    header = open(os.path.join(ROOT, "include", "pi.h")).read()
    assert L.pi_abi_version() == int(re.search(r"#define PI_ABI_VERSION (\d+)", header).group(1))
    # the binding's constants mirror the header's
    for name in ("PI_NDIAG", "PI_NWORK", "PI_NTAB"):
        assert getattr(binding, name) == int(re.search(r"#define %s (\d+)" % name, header).group(1))
    m = re.search(r"enum \{ PI_SRC_POINT = (\d+), PI_SRC_PLANE = (\d+) \}", header)
    assert (binding.PI_SRC_POINT, binding.PI_SRC_PLANE) == (int(m.group(1)), int(m.group(2)))
    # the descriptor's field order and types as the header declares them
    body = re.search(r"typedef struct \{(.*?)\} pi_grid_desc;", header, re.S).group(1)
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
    decl = re.findall(r"(int32_t|double)\s+(\w+)((?:\[[^\]]+\])*);", body)
    ctype = {"int32_t": C.c_int32, "double": C.c_double}
    max_src = int(re.search(r"#define PI_MAX_SRC (\d+)", header).group(1))
    assert binding.PI_MAX_SRC == max_src

    def arr(t, dims):
        ty = ctype[t]
        for k in reversed(re.findall(r"\[([^\]]+)\]", dims)):
            ty = ty * int(eval(k.replace("PI_MAX_SRC", str(max_src))))
        return ty

    want = [(n, arr(t, dims)) for t, n, dims in decl]
    got = [(n, t) for n, t in binding.GridDesc._fields_]
    assert [n for n, _ in want] == [n for n, _ in got]
    for (n, a), (_, b) in zip(want, got):
        assert C.sizeof(a) == C.sizeof(b) and getattr(a, "_type_", a) == getattr(b, "_type_", b), n


def test_descriptor_validation_rejects_bad_input():
    spec = synth.cfg1()
    base = binding.desc_from_spec(spec)
    f = binding.Fields()
    for k in ("nH", "x", "tau", "x_half", "tau_half", "E", "E_half"):
        setattr(f, k, 0x1000)   # never dereferenced: validation fails first
    cases = []
    for field, value in (("dx", -1.0), ("Q", -5.0), ("sigma0", 0.0), ("n_sub", 0), ("n_sub", 99),
                         ("weights", 7), ("precision", 9), ("spectrum", 3), ("thermal", 4)):
        d = binding.desc_from_spec(spec)
        setattr(d, field, value)
        cases.append(d)
    d = binding.desc_from_spec(spec)
    d.src[0] = 40
    cases.append(d)
    d = binding.desc_from_spec(spec)
    d.n[1] = 0
    cases.append(d)
    d = binding.desc_from_spec(spec)
    d.K[3] = -1.0
    cases.append(d)
    # a zero factor of eq. (4) would give dt = 0: the clock could never advance
    d = binding.desc_from_spec(spec)
    d.K[3] = 0.0
    cases.append(d)
    d = binding.desc_from_spec(spec)
    d.source = 2
    cases.append(d)
    # several sources: count, vertices, Q, and point sources only
    for nsrc, v, q, src in ((5, 0, 1.0, 0), (2, 33, 1.0, 0), (2, 0, -1.0, 0), (2, 0, 1.0, 1)):
        d = binding.desc_from_spec(spec)
        d.nsrc, d.src_more[0][:], d.Q_more[0], d.source = nsrc, (v, 0, 0), q, src
        cases.append(d)
    for d in cases:
        h = C.c_void_p()
        st = binding.lib().pi_grid_create(C.byref(d), C.byref(f), C.byref(h))
        assert st == binding.PI_EINVAL
        assert h.value is None
        assert len(binding.lib().pi_last_error()) > 0
    f2 = binding.Fields()
    h = C.c_void_p()
    assert binding.lib().pi_grid_create(C.byref(base), C.byref(f2), C.byref(h)) == binding.PI_EINVAL


def test_null_handles_are_rejected():
    L = binding.lib()
    assert L.pi_raytrace(None, 0, 0, None) == binding.PI_EINVAL
    assert L.pi_step_o2(None, 1.0, None) == binding.PI_EINVAL
    assert L.pi_grid_destroy(None) == binding.PI_OK


def test_library_table_matches_oracle_table(oracle_lib):
    """Two independent quadratures of the same blackbody integrals."""
    import oracle
    for T_bb, Q in ((1e5, 1e48), (3.75e4, 5e48)):
        a = binding.table_build(T_bb, Q)
        b = oracle.table_build(T_bb, Q)
        np.testing.assert_allclose(a[0], b[0], rtol=1e-14)
        np.testing.assert_allclose(a[1:], b[1:], rtol=1e-10, atol=0)


def test_request_struct_matches_header():
    header = open(os.path.join(ROOT, "include", "pi.h")).read()
    body = header.split("} pi_request;")[0].rsplit("typedef struct {", 1)[1]
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
    names = re.findall(r"\b(\w+)\s*;", body)
    assert names == [n for n, _ in binding.Request._fields_]


@pytest.mark.parametrize("precision", ["fp64", "fp32", "mixed"])
@pytest.mark.parametrize("kind", ["cfg1", "cfg2", "sources"])
def test_required_bytes(precision, kind):
    """pi_grid_required_bytes: the caller's fields are the arrays the Python
    layer allocates for the grid (counted here from numpy shapes, not from the
    library's formula); the library's own device bytes grow with the cells and
    include the re-solve list (one 8-byte entry per cell) only in mixed
    precision."""
    spec = {"cfg1": synth.cfg1(n=(17, 13, 11), src=(5, 0, 11)),
            "cfg2": synth.cfg2(n=24),
            "sources": synth.cfg2(n=20).with_(more_sources=(((3, 4, 5), 1e47), ((20, 0, 7), 2e47)))}[kind]
    fb, wb = binding.required_bytes(spec, precision)
    w = 8 if precision == "fp64" else 4
    ns = 1 + len(spec.more_sources)
    arrays = [spec.shape] * 3 + [(ns,) + spec.shape] * 2    # nH, x, x_half, tau, tau_half
    if spec.thermal == "evolve":
        arrays += [spec.shape] * 2                            # E, E_half
    assert fb == sum(int(np.prod(a)) for a in arrays) * w
    assert wb > 0
    big = spec.with_(n=tuple(2 * v for v in spec.n), src=tuple(2 * v for v in spec.src),
                     more_sources=tuple(((2 * a, 2 * b, 2 * c), q) for (a, b, c), q in spec.more_sources))
    assert binding.required_bytes(big, precision)[1] > wb
    if precision == "mixed":
        assert wb - binding.required_bytes(spec, "fp32")[1] == 8 * spec.ncells + 12


def test_required_bytes_rejects_bad_descriptor():
    d = binding.desc_from_spec(synth.cfg1())
    d.dx = -1.0
    a, b = C.c_size_t(), C.c_size_t()
    assert binding.lib().pi_grid_required_bytes(C.byref(d), C.byref(a), C.byref(b)) == binding.PI_EINVAL
