"""CPU checks of the C ABI: the library loads and exports every declared symbol."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", h) for h in ("hmg.h", "hmg_nn.h")]


def declared_symbols():
    names = set()
    for h in HEADERS:
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names |= set(re.findall(r"\b(hmg_[a-z_0-9]+)\s*\(", text))
    return sorted(names)


def test_header_declares_the_boundary():
    names = declared_symbols()
    for core in ("hmg_set_density", "hmg_solve_cases", "hmg_elastic_tensor", "hmg_sensitivity",
                 "hmg_oc_update"):
        assert core in names


def test_library_exports_every_declared_symbol():
    from paper_2301_08911_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("libhmg.so is not built; run python -m paper_2301_08911_amd.build")
    lib = ctypes.CDLL(_lib.LIB_PATH)
    missing = [s for s in declared_symbols() if not hasattr(lib, s)]
    assert not missing, missing
    assert set(_lib.SYMBOLS) == set(declared_symbols())


def test_config_struct_layout_matches_header(tmp_path):
    """The ctypes mirror of hmg_config has the C compiler's size and offsets."""
    import shutil
    import subprocess
    from paper_2301_08911_amd import _lib
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    fields = [f for f, _ in _lib.HmgConfig._fields_]
    prog = tmp_path / "layout.c"
    prog.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "%s"\nint main(void){\n'
                    'printf("%%zu", sizeof(hmg_config));\n%s\nreturn 0;}\n' % (
                        HEADERS[0], "".join('printf(" %%zu", offsetof(hmg_config, %s));' % f
                                        for f in fields)))
    exe = tmp_path / "layout"
    subprocess.run([cc, str(prog), "-o", str(exe)], check=True)
    out = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True,
                                          check=True).stdout.split()]
    assert out[0] == ctypes.sizeof(_lib.HmgConfig)
    assert out[1:] == [getattr(_lib.HmgConfig, f).offset for f in fields]


def test_no_fallback_when_library_missing(tmp_path, monkeypatch):
    from paper_2301_08911_amd import _lib
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "absent.so"))
    monkeypatch.setattr(_lib, "_lib", None)
    with pytest.raises(ImportError):
        _lib.load()


@pytest.mark.parametrize("nu", [0.3, 0.0, 0.45, -0.5])
def test_library_element_constants_match_the_oracle(nu):
    """The library's K0 (exact 1D integrals) and load template against the
    oracle's (2x2x2 Gauss quadrature); host-only, so it runs without a GPU."""
    import numpy as np
    from oracle import hmgref as O
    from paper_2301_08911_amd import _lib
    lib = _lib.load()
    K0 = np.zeros(576)
    load = np.zeros(144)
    dp = ctypes.POINTER(ctypes.c_double)
    lam0 = ctypes.c_double()
    msig = np.zeros(8 * 576)
    st = lib.hmg_element_constants(nu, K0.ctypes.data_as(dp), load.ctypes.data_as(dp),
                                   ctypes.byref(lam0), msig.ctypes.data_as(dp))
    assert st == 0
    K0o = O.element_stiffness(1.0, nu)
    assert np.abs(K0.reshape(24, 24) - K0o).max() < 1e-14 * np.abs(K0o).max()
    ref = O.unit_strain_displacements() @ K0o            # (6, 24) = (K0 chi^i)^T
    assert np.abs(load.reshape(6, 24) - ref).max() < 1e-14 * np.abs(K0o).max()
    # spectral bound: largest eigenvalue of K0 v = lambda blockdiag(K0) v
    from scipy.linalg import eigh
    Bd = np.zeros((24, 24))
    for a in range(8):
        Bd[3 * a:3 * a + 3, 3 * a:3 * a + 3] = K0o[3 * a:3 * a + 3, 3 * a:3 * a + 3]
    lam = eigh(K0o, Bd, eigvals_only=True).max()
    assert abs(lam0.value - lam) < 1e-6 * lam, (lam0.value, lam)
    # sub-element Galerkin matrices: W_sigma read off the oracle's prolongation
    # (fine 8^3 from coarse 4^3, coarse element at (1,1,1), no wrap), and their
    # sum is the stiffness of the 2h element, 2 K0 in 3D
    msig = msig.reshape(8, 24, 24)
    P = O.prolongation((8, 8, 8)).tocsr()
    scale = np.abs(K0o).max()
    for sg in range(8):
        s0, s1, s2 = sg & 1, (sg >> 1) & 1, (sg >> 2) & 1
        W = np.zeros((8, 8))
        for b in range(8):
            fx, fy, fz = 2 + s0 + (b & 1), 2 + s1 + ((b >> 1) & 1), 2 + s2 + ((b >> 2) & 1)
            for A in range(8):
                cx, cy, cz = 1 + (A & 1), 1 + ((A >> 1) & 1), 1 + ((A >> 2) & 1)
                W[b, A] = P[3 * (fx + 8 * (fy + 8 * fz)), 3 * (cx + 4 * (cy + 4 * cz))]
        assert np.allclose(W.sum(axis=1), 1.0, atol=1e-15)
        W3 = np.kron(W, np.eye(3))
        assert np.abs(msig[sg] - W3.T @ K0o @ W3).max() < 1e-14 * scale, sg
    assert np.abs(msig.sum(axis=0) - 2.0 * K0o).max() < 1e-14 * scale


def test_library_element_constants_refuse_bad_arguments():
    import numpy as np
    from paper_2301_08911_amd import _lib
    lib = _lib.load()
    K0 = np.zeros(576)
    dp = ctypes.POINTER(ctypes.c_double)
    assert lib.hmg_element_constants(0.5, K0.ctypes.data_as(dp), None, None, None) == 1
    assert lib.hmg_element_constants(-1.0, K0.ctypes.data_as(dp), None, None, None) == 1
    assert lib.hmg_element_constants(0.3, None, None, None, None) == 1
    assert lib.hmg_element_constants(0.3, K0.ctypes.data_as(dp), None, None, None) == 0
