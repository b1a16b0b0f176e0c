"""bq_batch_set_static: the batch set-up that allocates no device memory
(tables in the library's static per-device array), through the C ABI,
against bq_batch_set with the same members.  Results must be bitwise equal
(the kernels and their arithmetic are the same; only the address of the
tables differs)."""
import numpy as np
import pytest

from paper_1909_04153_amd import scenarios as S

pytestmark = pytest.mark.gpu

FIELDS = ("eta", "P", "Q")


@pytest.fixture(scope="module")
def bq():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    from paper_1909_04153_amd import bq as m

    m.load()
    return m


def _specs():
    return [S.sloping_beach(nx=200, ny=40, dx=0.1, x_toe=2.0, t_end=0.0),
            S.solitary_flat(nx=130, ny=70, x0=2.0),
            S.rip_beach_scaled(96, 72, cfl=0.125, fstar_order=1, t_end=0.0)]


def _fresh(bq, specs):
    return [bq.domain_from_spec(s, precision=bq.FP32) for s in specs]


def _advance(batch, doms, steps):
    batch.step(steps)
    batch.sync()
    out = []
    for d in doms:
        i = d.sync()
        assert i.status == 0 and i.n == steps, i
        out.append([d.read(f) for f in FIELDS])
    return out


def test_static_tables_match_allocated_tables(bq):
    specs = _specs()
    # the batch under test is created on one member, then set (without
    # allocation) to three members, then to a single smaller member
    seed = _fresh(bq, specs[2:])
    st = bq.Batch(seed, lanes=2)
    ref = bq.Batch(_fresh(bq, specs[2:]), lanes=2)
    st.set_graph_steps(4)
    ref.set_graph_steps(4)
    for members in (specs, specs[2:]):
        a, b = _fresh(bq, members), _fresh(bq, members)
        before = bq.live_handles()
        st.set(a, static=True)
        # no stream, event or graph executable was made by the call
        assert bq.live_handles() == before
        ref.set(b)
        assert st.lanes == ref.lanes == min(2, len(members))
        got, want = _advance(st, a, 9), _advance(ref, b, 9)
        for g, w, s in zip(got, want, members):
            for f, x, y in zip(FIELDS, g, w):
                assert np.array_equal(x, y), (s["name"], f)
    st.close()
    ref.close()


def test_static_tables_ownership_and_size_limit(bq):
    specs = _specs()
    d1, d2 = _fresh(bq, specs[:1]), _fresh(bq, specs[1:2])
    b1, b2 = bq.Batch(d1, lanes=1), bq.Batch(d2, lanes=1)
    b1.set(d1, static=True)
    b1.step(2)
    # b2 takes the device's static array: b1 must set its members again
    b2.set(d2, static=True)
    with pytest.raises(bq.BqError) as e:
        b1.step(1)
    assert e.value.code == bq.ESTATE
    b2.step(2)
    b1.set(d1)                      # back to its own (allocated) tables
    b1.step(1)
    b1.sync()
    b2.sync()
    assert d1[0].sync().n == 3 and d2[0].sync().n == 2
    # a member list whose tables exceed the array is refused on the host and
    # leaves the batch as it was
    many = d2 * 20000
    with pytest.raises(bq.BqError) as e:
        b2.set(many, static=True)
    assert e.value.code == bq.EINVAL
    b2.step(1)
    b2.sync()
    assert d2[0].sync().n == 3
    b1.close()
    b2.close()
