"""lf_exact_sum_noalloc against lf_debug_exact_sum through the C ABI (needs a GPU).

The entry point uses the library's fixed device scratch instead of allocating.  Two
calls in a row, the second on a smaller input, must each give exactly what the
allocating entry point gives on the same values (and the exactly rounded sum), and sizes
beyond the stated maximum are refused before anything runs.
"""
import math
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def env():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2210_03211_amd as lf
    lf.load_library()
    h = lf.Handle(0)
    yield torch, lf, h
    h.close()


def test_noalloc_equals_allocating_entry_point(env):
    torch, lf, h = env
    rng = np.random.default_rng(21)
    for n in (300_001, 4_097):                     # the second call is smaller
        v = 2.0 ** rng.uniform(-60, 20, n) * np.where(rng.random(n) < 0.5, -1, 1)
        vd = torch.from_numpy(v).cuda()
        say("noalloc", n)
        a = h.lf_exact_sum_noalloc(vd)
        b = h.lf_debug_exact_sum(vd)
        assert a == b == math.fsum(v.tolist())
    # a second handle on the same device shares the scratch; results stay exact
    h2 = lf.Handle(0)
    v = rng.random(1000)
    say("noalloc second handle", v.size)
    assert h2.lf_exact_sum_noalloc(torch.from_numpy(v).cuda()) == math.fsum(v.tolist())
    assert h2.lf_exact_sum_noalloc(torch.zeros(0, dtype=torch.float64, device="cuda")) == 0.0
    h2.close()


def test_noalloc_errors(env):
    torch, lf, h = env
    with pytest.raises(lf.LazyFoxError):               # out of the accumulator's value range
        h.lf_exact_sum_noalloc(torch.tensor([2.0 ** 40], dtype=torch.float64).cuda())
    # the flag is cleared again for the next call
    assert h.lf_exact_sum_noalloc(torch.tensor([1.5, 2.25], dtype=torch.float64).cuda()) == 3.75
    # a size beyond the maximum is refused on the host, before any device access
    vd = torch.zeros(1, dtype=torch.float64, device="cuda")
    with pytest.raises(lf.LazyFoxError) as e:
        h._noalloc_raw(vd, (1 << 40) + 1)
    assert e.value.code == lf.LF_EINVAL
