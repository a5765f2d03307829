"""C ABI checks that need no GPU: the library loads, exports every declared entry
point, and rejects invalid arguments before touching the device."""
import ctypes as ct
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "qfdtd.h")


def header_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    names = set(re.findall(r"\b(qfdtd_[a-z_]+)\s*\(", txt))
    return sorted(n for n in names if not n.endswith("_fn"))


@pytest.fixture(scope="module")
def L():
    from paper_2211_10185_amd import _lib
    return _lib


def test_every_declared_symbol_is_exported(L):
    names = header_functions()
    assert len(names) >= 15
    for n in names:
        assert hasattr(L.lib, n), n
    assert set(names) == set(L.exported_symbols())


def _create(L, N=32, a=0.25, m=1.0, kin=1, vkind=1, prec=0, k=3, sectors=None, K=0, knots=None):
    pot = L.Potential()
    pot.kind = vkind
    pot.p[0] = 1.0
    keep = []
    if knots is not None:
        kn = np.ascontiguousarray(knots, dtype=np.float64)
        keep.append(kn)
        pot.knots = kn.ctypes.data_as(ct.POINTER(ct.c_double))
        pot.n_knots = kn.shape[0]
    opt = L.Options()
    opt.precision = prec
    opt.n_states = k
    opt.measure_every = K
    if sectors is not None:
        sec = (ct.c_int32 * k)(*sectors)
        keep.append(sec)
        opt.sectors = ct.cast(sec, ct.POINTER(ct.c_int32))
    ctx = ct.c_void_p()
    st = L.lib.qfdtd_create(ct.byref(ctx), N, a, m, kin, ct.byref(pot), ct.byref(opt))
    return st, ctx


@pytest.mark.parametrize("N,kin,code", [(31, 1, -2), (6, 1, -2), (14, 1, -2), (7 * 8, 2, -2), (288, 1, -2),
                                        (514, 0, -2), (44, 3, -2)])
def test_unsupported_lattice_sizes(L, N, kin, code):
    st, ctx = _create(L, N=N, kin=kin)
    assert st == code
    assert not ctx.value
    assert L.lib.qfdtd_last_error(None)


@pytest.mark.parametrize("kw", [dict(a=0.0), dict(m=-1.0), dict(kin=4), dict(vkind=9), dict(prec=2),
                                dict(k=0), dict(k=9), dict(sectors=[0, 7, 0]), dict(K=-1),
                                dict(vkind=0), dict(vkind=4, knots=np.array([[0, 1], [1, 2.0]])),
                                dict(vkind=4, knots=np.array([[0, 1], [2, 2.0], [1, 3.0]]))])
def test_invalid_arguments(L, kw):
    st, ctx = _create(L, **kw)
    assert st == -1
    assert not ctx.value


def test_null_context_calls(L):
    assert L.lib.qfdtd_evolve(None, 10, 0.01) == -1
    assert L.lib.qfdtd_set_state(None, 0, None) == -1
    assert L.lib.qfdtd_states(None, 1, None, None) == -1
    L.lib.qfdtd_destroy(None)


def test_footprint_scales_with_volume(L):
    f1 = L.lib.qfdtd_footprint(64, 1, 0, 3)
    f2 = L.lib.qfdtd_footprint(128, 1, 0, 3)
    assert 7.5 < f2 / f1 < 8.5
    assert L.lib.qfdtd_footprint(128, 1, 1, 3) > f2
    assert L.lib.qfdtd_footprint(0, 1, 0, 3) == 0


def test_potential_files_round_trip_in_every_format(tmp_path):
    from paper_2211_10185_amd.solver import read_potential_file, write_potential_file
    N = 5
    g = np.random.default_rng(3)
    V = g.standard_normal((N, N, N)) * 7 + 1j * g.standard_normal((N, N, N))
    # library writer -> library reader: the same doubles
    write_potential_file(tmp_path / "w.txt", V)
    assert np.array_equal(read_potential_file(tmp_path / "w.txt", N), V)
    i = np.indices((N, N, N)).reshape(3, -1).T
    vr, vi = V.real.ravel(), V.imag.ravel()
    perm = g.permutation(N ** 3)
    forms = {
        "re.txt": (np.column_stack([vr]), V.real),
        "reim.csv": (np.column_stack([vr, vi]), V),
        "idx_re.txt": (np.column_stack([i, vr])[perm], V.real),
        "idx_reim.txt": (np.column_stack([i, vr, vi])[perm], V),
    }
    for name, (rows, want) in forms.items():
        sep = "," if name.endswith(".csv") else " "
        with open(tmp_path / name, "w") as f:
            f.write("# header line\n\n")
            for r in rows:
                f.write(sep.join(repr(float(x)) for x in r) + "  # trailing comment\n")
        got = read_potential_file(tmp_path / name, N)
        assert np.array_equal(got, want.astype(np.complex128)), name


@pytest.mark.parametrize("content,what", [
    ("1 2\n3\n", "inconsistent"),
    ("1 2 3\n", "fields"),
    ("abc\n", "bad number"),
    ("", "no records"),
    ("0 0 0 1\n0 0 0 2\n", "twice"),
    ("0 0 9 1\n", "range"),
    ("1\n" * 7, "records"),
    ("nan 0\n" * 8, "non-finite"),
])
def test_potential_file_errors(tmp_path, content, what, L):
    from paper_2211_10185_amd.solver import read_potential_file
    p = tmp_path / "bad.txt"
    p.write_text(content)
    with pytest.raises(L.QfdtdError) as ei:
        read_potential_file(p, 2)
    assert ei.value.status == L.E_INVALID
    assert what in str(ei.value), str(ei.value)
    with pytest.raises(L.QfdtdError):
        read_potential_file(tmp_path / "missing.txt", 2)


def test_dft_stage_library_exports_its_header():
    from paper_2211_10185_amd import dft_stage as D
    txt = re.sub(r"/\*.*?\*/", "", open(os.path.join(ROOT, "include", "dft_stage.h")).read(), flags=re.S)
    names = sorted(set(re.findall(r"\b(dft16_[a-z_]+)\s*\(", txt)))
    assert names == D.exported_symbols()
    for n in names:
        assert hasattr(D.lib, n), n


def test_dft_stage_rejects_invalid_arguments_before_the_device():
    from paper_2211_10185_amd import dft_stage as D
    L = D.lib
    assert L.dft16_stage_run(7, 1, 1, 256, 1, None) == -1          # unknown variant
    assert L.dft16_stage_run(0, None, 1, 256, 1, None) == -1       # NULL input
    assert L.dft16_stage_run(0, 1, 1, 100, 1, None) == -1          # not a multiple of 256
    assert L.dft16_stage_run(1, 1, 1, 256, 0, None) == -1          # reps < 1
    ms = ct.c_double()
    assert L.dft16_stage_time(0, 1, 1, 256, 1, 0, None, ct.byref(ms)) == -1
    assert b"iters" in L.dft16_stage_last_error()
