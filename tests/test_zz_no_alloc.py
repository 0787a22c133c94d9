"""The decoupling entry point that allocates nothing (cptr_decouple_noalloc)
against the allocating one (cptr_decouple), through the C ABI: the same
kernels, so the scaled matrix and right-hand side agree bit for bit; two
calls in a row with the second on a smaller system (the shared scratch keeps
the first call's contents, so stale weights or a stale singular-cell word
would show); the size limit and the singular-block error."""
import ctypes

import numpy as np
import pytest

import oracle as O
from synthetic import config3, tiny

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():   # collected on CPU-only machines but never run there
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_1912_04385_amd import cptr  # noqa: E402


def _dev(s):
    return (torch.from_numpy(s.row_ptr).cuda(), torch.from_numpy(s.col_idx).cuda(),
            torch.from_numpy(s.vals.reshape(-1)).cuda(), torch.from_numpy(s.rhs).cuda())


def _both(s, variant):
    rp, ci, v, r = _dev(s)
    ref_abar, ref_rb = cptr.decouple(variant, rp, ci, v, r)
    abar = torch.full_like(v, np.nan)
    rb = torch.full_like(r, np.nan)
    cptr.decouple_noalloc(variant, rp, ci, v, r, abar, rb)
    return ref_abar.cpu().numpy(), ref_rb.cpu().numpy(), abar.cpu().numpy(), rb.cpu().numpy()


@pytest.mark.parametrize("variant", [cptr.VARIANT_CPTR3, cptr.VARIANT_CPR, cptr.VARIANT_CPTR])
def test_noalloc_matches_allocating_entry_point_twice(variant):
    big = config3(1, 300, 200)                 # 60k cells, b = 8
    small = tiny(13, 9, 6, peclet=2.0, seed=4)   # then a smaller system, b = 6
    for s in (big, small):
        print(f"case decouple_noalloc variant={variant} n={s.n} b={s.b}", flush=True)
        ra, rr, a, r = _both(s, variant)
        assert np.array_equal(a, ra) and np.array_equal(r, rr)
    # and against the oracle's decoupling on the small one
    ref = O.decouple(O.bsr_of(small), small.rhs, variant=variant)
    assert np.array_equal(a, ref.Abar.vals.reshape(-1)) and np.array_equal(r, ref.rhsbar)


def test_noalloc_size_limit_is_rejected_before_any_kernel():
    print("case decouple_noalloc size limit", flush=True)
    s = tiny(4, 3, 8, seed=0)
    rp, ci, v, r = _dev(s)
    n = 700_000                              # needs 2 * 44.8 MB + 5.6 MB of scratch
    rc = cptr.lib().cptr_decouple_noalloc(0, n, 8, cptr._ptr(rp), cptr._ptr(ci), cptr._ptr(v), cptr._ptr(r), 0, 1,
                                          cptr._ptr(v), cptr._ptr(r), cptr._stream())
    assert rc == -1 and b"scratch" in cptr.lib().cptr_last_error()


def test_noalloc_singular_block_then_a_good_call():
    print("case decouple_noalloc singular block", flush=True)
    s = tiny(6, 5, 4, seed=1)
    rows = np.repeat(np.arange(s.n), np.diff(s.row_ptr))
    e = np.nonzero((rows == 13) & (s.col_idx == 13))[0][0]
    s.vals[e, 2:, 2:] = 0.0
    rp, ci, v, r = _dev(s)
    abar, rb = torch.empty_like(v), torch.empty_like(r)
    with pytest.raises(cptr.CptrError) as err:
        cptr.decouple_noalloc(0, rp, ci, v, r, abar, rb)
    assert err.value.status == -3 and "cell 13" in str(err.value)
    # the singular-cell word is cleared by the next call
    good = tiny(6, 5, 4, seed=1)
    ra, rr, a, r2 = _both(good, 0)
    assert np.array_equal(a, ra) and np.array_equal(r2, rr)
