"""Host-only checks of the C-ABI library: it loads, exports every function that
include/ace.h declares, and rejects invalid problems before touching a GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ace.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ace_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def ace():
    from paper_2312_07010_amd import ace as A
    return A


def test_library_exports_every_declared_function(ace):
    names = declared_functions()
    assert len(names) >= 30
    L = ace.lib()
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing
    # the binding wraps exactly the declared calls
    assert set(ace._SIGS) == set(names)


def test_strerror_and_version(ace):
    for code in range(-8, 5):
        assert ace.strerror(code)
    assert b"gfx950" in ace.lib().ace_version()


def _create(ace, d, N, L, R, eps, dt, bc):
    L_ = ace.lib()
    n = (ctypes.c_int64 * 3)(*(list(N) + [1] * (3 - len(N))))
    lo = (ctypes.c_double * 3)(*(list(L) + [0.0] * (3 - len(L))))
    hi = (ctypes.c_double * 3)(*(list(R) + [1.0] * (3 - len(R))))
    h = ctypes.c_void_p()
    return L_.ace_create(d, n, lo, hi, eps, dt, bc, ctypes.byref(h))


@pytest.mark.parametrize("args,code", [
    ((0, [8], [0], [1], 0.1, 1e-3, 0), -1),          # d out of range
    ((4, [8] * 3, [0] * 3, [1] * 3, 0.1, 1e-3, 0), -1),
    ((1, [8], [1], [0], 0.1, 1e-3, 0), -1),          # L >= R
    ((1, [8], [0], [1], 0.0, 1e-3, 0), -1),          # eps <= 0
    ((1, [8], [0], [1], float("nan"), 1e-3, 0), -1),
    ((1, [8], [0], [1], 0.1, 1e-3, 7), -1),          # unknown BC
    ((1, [0], [0], [1], 0.1, 1e-3, 0), -2),          # HN needs N >= 1
    ((1, [1], [0], [1], 0.1, 1e-3, 1), -2),          # HD needs N >= 2
    ((1, [2], [0], [1], 0.1, 1e-3, 2), -2),          # P needs N >= 3
    ((2, [8, 9], [0, 0], [1, 1], 0.1, 1e-3, 0), -3),  # anisotropic spacing
    ((1, [8], [0], [1], 0.1, 0.0, 0), -4),           # dt <= 0
    ((1, [8], [0], [1], 0.1, 2.0, 0), -4),           # dt >= 2: cubic not monotone
])
def test_create_rejects_invalid_problems(ace, args, code):
    assert _create(ace, *args) == code


def test_monitor_status_reports_every_warning(ace):
    """The check ace_run_monitored applies to its monitor series (Theorem 2:
    the max-norm stays <= 1; Theorem 3: the energy does not rise), fed with
    synthetic series: each warning alone, both together (both bits, the
    max-principle code returned), none without the step conditions, and
    non-finite values."""
    u = 2.0 ** -53
    W_MP, W_EU = ace.ACE_W_MAXPRINCIPLE, ace.ACE_W_ENERGY_UP
    b_mp, b_eu = ace.warn_bit(W_MP), ace.warn_bit(W_EU)
    E_down = [3.0, 2.0, 1.0]
    E_up = [3.0, 2.0, 2.0 + 3e-14 * 2.0]
    m_ok = [1.0, 1.0 + 4 * u, 0.5]
    m_bad = [1.0, 1.0 + 8 * u, 0.5]
    assert ace.monitor_status(E_down, m_ok) == (ace.ACE_OK, 0)
    assert ace.monitor_status(E_down, m_bad) == (W_MP, b_mp)
    assert ace.monitor_status(E_up, m_ok) == (W_EU, b_eu)
    assert ace.monitor_status(E_up, m_bad) == (W_MP, b_mp | b_eu)
    # a rise within the 1e-14 relative slack is rounding, not a violation
    assert ace.monitor_status([1.0, 1.0 + 5e-15], [1.0, 1.0]) == (ace.ACE_OK, 0)
    # outside the step conditions the theorems promise nothing
    assert ace.monitor_status(E_up, m_bad, conditions_ok=False) == (ace.ACE_OK, 0)
    assert ace.monitor_status([1.0, float("nan")], [1.0, 1.0])[0] == ace.ACE_E_NONFINITE
    assert ace.monitor_status([1.0, 1.0], [1.0, float("inf")])[0] == ace.ACE_E_NONFINITE
    assert ace.monitor_status([], [])[0] == ace.ACE_E_ARG
