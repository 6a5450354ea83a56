"""The streaming probe behind the bench line's ceilings (lbm_stream_probe):
it runs, gives a time that a real memory system can deliver, and rejects bad
arguments."""
import math

import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import paper_1909_13086_amd as P
    return P


@pytest.mark.parametrize("pattern", [0, 1], ids=["in_place", "two_lattices"])
def test_probe_times_are_physical(P, pattern):
    nbytes = 64 << 20
    print(f"case stream probe {nbytes} bytes pattern {pattern}", flush=True)
    with P.Context(device=0, max_slots=1) as ctx:
        us = ctx.stream_probe(nbytes, pattern, 20)
    assert math.isfinite(us) and us > 0
    # 2 x 64 MiB per launch cannot move faster than 20 TB/s
    assert 2 * nbytes / (us * 1e-6) < 20e12


def test_probe_rejects_bad_arguments(P):
    with P.Context(device=0, max_slots=1) as ctx:
        for args in ((100, 1, 4), (1 << 20, 7, 4), (1 << 20, 1, 0)):
            with pytest.raises(P.LbmError):
                ctx.stream_probe(*args)
