"""The allocation-free pair histogram (rbsog_rdf_counts_noalloc) through the C
ABI against rbsog_rdf_counts, which allocates its device histogram per call:
integer counts, so bit-exact, on two calls in a row of which the second is
smaller (fewer bins, then a smaller system), so counts of an earlier call
left in the shared static array would show."""
from __future__ import annotations

import sys

import numpy as np
import pytest

from paper_2512_24970_amd import rbsog as R
from paper_2512_24970_amd import workloads as W

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def gpu_system(cfg, precision=R.FP64, **over):
    import torch
    sysp = dict(cfg["sys"], **over)
    ctx = R.Context(0)
    p = R.make_params(sysp, precision, n_atoms=len(cfg["types"]))
    dev = torch.device("cuda", 0)
    ctx.rbsog_set_system(p, torch.as_tensor(cfg["types"], device=dev), torch.as_tensor(cfg["pos"], device=dev),
                         torch.as_tensor(cfg["vel"], device=dev))
    return ctx


def test_noalloc_rdf_equals_allocating_rdf():
    _say("case: allocation-free rdf, nacl_512 then smaller calls")
    a = gpu_system(W.config("nacl_512"))
    ref1 = a.rbsog_rdf_counts(10.0, 400)
    got1 = a.rbsog_rdf_counts_noalloc(10.0, 400)
    assert ref1.sum() > 0
    assert np.array_equal(got1, ref1)
    # second call, smaller: fewer bins over a shorter range
    ref2 = a.rbsog_rdf_counts(6.0, 90)
    got2 = a.rbsog_rdf_counts_noalloc(6.0, 90)
    assert np.array_equal(got2, ref2)
    # a smaller system in another context on the same GPU, after some steps
    b = gpu_system(W.config("nacl_small"))
    b.rbsog_step(3, want_energy=False)
    ref3 = b.rbsog_rdf_counts(8.0, 60)
    got3 = b.rbsog_rdf_counts_noalloc(8.0, 60)
    assert ref3.sum() > 0
    assert np.array_equal(got3, ref3)


def test_noalloc_rdf_rejects_more_bins_than_the_scratch():
    _say("case: allocation-free rdf, oversized request")
    a = gpu_system(W.config("nacl_512"))
    with pytest.raises(R.RbsogError) as e:
        a.rbsog_rdf_counts_noalloc(10.0, 4097)  # 2 x 2 x 4097 > 16384 counters
    assert e.value.code == -1
    got = a.rbsog_rdf_counts_noalloc(10.0, 4096)  # exactly the maximum
    assert np.array_equal(got, a.rbsog_rdf_counts(10.0, 4096))
