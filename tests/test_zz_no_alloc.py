"""The allocation-free entry point gd_reshuffle_neighbors_static against
gd_reshuffle_neighbors, through the C ABI: two calls in a row on one GPU (the
second with a smaller input, over the table the first one left), each
relabelling identical rows identically, bit for bit."""
import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2609_35967_amd import Engine, load  # noqa: E402


@pytest.mark.parametrize("k", [32, 20])
def test_static_reshuffle_matches_workspace_form(k):
    load()
    for call, (n, refresh) in enumerate([(6000, 3), (2500, 4)]):  # the second call is smaller
        params = workloads.const_box_params(n, k=k)
        st = workloads.const_box(40 + call, n)
        st["M"] = st["M"].copy()
        st["M"][::11] = 0.0  # inactive particles: N < n
        eng = Engine(params, st, seed=77)
        eng.build_neighbors()
        torch.cuda.synchronize()
        before = eng.nbr.clone()
        eng.reshuffle_neighbors(refresh)
        torch.cuda.synchronize()
        want = eng.nbr.clone()
        eng.nbr.copy_(before)
        torch.cuda.synchronize()
        eng.reshuffle_neighbors_static(refresh)
        torch.cuda.synchronize()
        got = eng.nbr.cpu().numpy()
        assert np.array_equal(got, want.cpu().numpy()), f"call {call}"
        # and both are the oracle's relabelling
        N = int(eng.n_active.item())
        ref = oracle.reshuffle(before.cpu().numpy(), eng.cnt.cpu().numpy(), N, 77, refresh)
        assert np.array_equal(got, ref)
        assert eng.status() & ~0x4 == 0
