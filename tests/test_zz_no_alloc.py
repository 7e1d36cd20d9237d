"""The allocation-free entry point (wcsph_export_neighbour_lists_noalloc)
against the entry point it is a variant of (wcsph_export_neighbour_lists),
through the C ABI: equal lists on two calls in a row, the second on a
smaller context, and the size limit of its scratch array."""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

wc = pytest.importorskip("paper_2609_05494_amd")


def _same_lists(a, b):
    assert len(a) == len(b)
    for k, (u, v) in enumerate(zip(a, b)):
        assert np.array_equal(np.sort(u), np.sort(v)), k


def test_noalloc_lists_equal_the_allocating_entry_point():
    first = wc.Solver(workloads.C1(), "cuda:0")
    first.step(40)
    print("[gpu] no-alloc export: C1 after 40 steps", flush=True)
    ref = first.export_neighbour_lists()
    got = first.export_neighbour_lists(noalloc=True)
    _same_lists(got, ref)
    assert sum(len(x) for x in got) > 15 * first.nf  # about twenty neighbours each
    # the state is untouched: the run continues as without the exports
    first.step(10)
    _, fa = first.fluid()
    other = wc.Solver(workloads.C1(), "cuda:0")
    other.step(50)
    _, fb = other.fluid()
    for u, v in zip(fa, fb):
        assert np.array_equal(u, v)
    other.close()
    first.close()
    # a second call on a smaller context: the shared array keeps the last
    # call's contents, so the counts must have been cleared
    small = wc.Solver(workloads.tiny(), "cuda:0")
    small.step(15)
    print("[gpu] no-alloc export: tiny after 15 steps", flush=True)
    got2 = small.export_neighbour_lists(noalloc=True)
    ref2 = small.export_neighbour_lists()
    _same_lists(got2, ref2)
    assert len(got2) == small.nf < 1000
    small.close()


def test_noalloc_rejects_a_context_beyond_its_array():
    cfg = workloads.base(0.200, 0.100, 1.0e-3, 4.0e-3, 600.0)  # 19,950 fluid > 16,131
    s = wc.Solver(cfg, "cuda:0")
    with pytest.raises(wc.WcsphError) as e:
        s.export_neighbour_lists(noalloc=True)
    assert e.value.status == wc.E_RANGE and "at most" in str(e.value)
    s.step(2)  # the context is unchanged and still usable
    s.close()
