"""GPU: the allocation-free recomputation (bss_green_from_field_noalloc,
scratch in the library's static device array) against the allocating entry
point bss_green_from_field, through the C ABI, on two calls in a row with the
second on a smaller field, and its size limit."""
import numpy as np
import pytest

import paper_1504_05090_amd as bss
from paper_1504_05090_amd.workloads import BASE_SEED, random_field

pytestmark = pytest.mark.gpu
T = 0.25


def test_noalloc_matches_the_allocating_entry_point():
    import torch
    s = torch.cuda.Stream()
    cases = [(16, 2.0, 20.0, 0.5, 8, 1), (8, 2.0, 10.0, 0.5, 10, 5)]   # the second input is smaller
    for L, U, beta, dtau, n_stab, l in cases:
        print(f"[gpu] noalloc L={L} beta={beta} n_stab={n_stab} l={l}", flush=True)
        f = torch.from_numpy(random_field(L, beta, dtau, BASE_SEED + L)).cuda()
        want = bss.green_from_field(L, U, T, beta, dtau, n_stab, l, f).cpu().numpy()
        with torch.cuda.stream(s):
            got = bss.green_from_field(L, U, T, beta, dtau, n_stab, l, f, stream=s, noalloc=True)
        s.synchronize()
        got = got.cpu().numpy()
        assert np.array_equal(got, want), float(np.max(np.abs(got - want)))


def test_noalloc_rejects_fields_beyond_its_scratch():
    import torch
    assert bss.lib().bss_green_from_field_noalloc_limit() == 12 << 20
    f = torch.ones((80, 400), dtype=torch.int8, device="cuda")
    with pytest.raises(bss.BssError) as e:
        bss.green_from_field(20, 2.0, T, 40.0, 0.5, 8, 1, f, noalloc=True)
    assert e.value.status == bss.BSS_E_UNSUPPORTED
