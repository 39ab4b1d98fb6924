"""Host-side checks of the GPU library (no GPU needed): the shared object
loads, exports every entry point that include/rbsog.h declares, and its
host-side SOG planning agrees with the oracle's independent solver."""
from __future__ import annotations

import ctypes as C
import os
import re

import numpy as np
import pytest

import oracle as O
from paper_2512_24970_amd import rbsog as R
from paper_2512_24970_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "rbsog.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rbsog_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    L = R.lib()
    names = _declared()
    assert len(names) >= 15
    for n in names:
        assert hasattr(L, n), n
    # and the binding covers them all
    assert set(names) <= set(R.ABI)


def test_version_string():
    assert b"librbsog" in R.lib().rbsog_version()


@pytest.mark.parametrize("eps,r_shell", [(1e-5, 10.0), (1e-5, 11.0), (1e-7, 10.0), (3e-4, 9.0)])
def test_sog_planning_matches_oracle(eps, r_shell):
    """The library's SOG solver (host C++) and the oracle's (C) are separate
    code for the same equations (eqs. 5, 7-10); they agree on b, M and the
    cutoff root to the conditioning of the root (dh/dx ~ 1e-5)."""
    lib = R.rbsog_sog_params(eps, r_shell)
    cfg = W.config("nacl_512")
    sysp = dict(cfg["sys"], sog_eps=eps, r_shell=r_shell)
    p = O.make_params(sysp)
    assert lib["b"] == p.b
    assert lib["M"] == p.M
    assert lib["x_c"] == pytest.approx(p.x_c, rel=1e-11)
    w = np.array(p.w[: p.M + 1])
    assert np.allclose(lib["w"], w, rtol=1e-10, atol=0)


def test_create_without_gpu_fails_cleanly():
    """On a machine without a GPU, rbsog_create returns an error code."""
    try:
        import torch
        if torch.cuda.is_available():
            pytest.skip("GPU present")
    except Exception:
        pass
    h = C.c_void_p()
    rc = R.lib().rbsog_create(C.byref(h), 0, None)
    assert rc != 0 and not h.value
