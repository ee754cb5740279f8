"""The optional finiteness check (rd_set_check_finite): a result holding NaN
or infinity is reported as RD_ENONFINITE by every entry point, a finite one
passes unchanged, and the check refuses to run inside a stream capture."""
import numpy as np
import pytest
import torch

import paper_1309_1720_amd as rd
import rd_inputs as ri
from rdtest import dev, host, problems

pytestmark = pytest.mark.gpu


@pytest.fixture
def checking():
    rd.set_check_finite(True)
    yield
    rd.set_check_finite(False)


def fk(nx=70, ny=40, nz=None, steps=3, **kw):
    stencil = "lap27" if nz else "lap9"
    w = ri.workload("fk_1024_rk4", nx=nx, ny=ny, stencil=stencil, **({"nz": nz} if nz else {}), **kw)
    _, pr = problems(w, nsteps=steps)
    z0 = ri.random_fields("fk", nx, ny, 5, nz=nz)
    return pr, z0


def poisoned(z0, value=np.nan):
    z = [a.copy() for a in z0]
    z[0].flat[17] = value
    return z


@pytest.mark.parametrize("nz", [None, 9])
def test_step_reports_nonfinite_and_passes_finite(checking, nz):
    pr, z0 = fk(nz=nz)
    ref = dev(z0)
    rd.set_check_finite(False)
    rd.step(pr, ref)
    rd.set_check_finite(True)
    z = dev(z0)
    rd.step(pr, z)  # finite: no error, same bits as the unchecked call
    assert all(np.array_equal(a, b) for a, b in zip(host(z), host(ref)))
    for bad in (np.nan, np.inf):
        with pytest.raises(rd.RDError) as e:
            rd.step(pr, dev(poisoned(z0, bad)))
        assert e.value.code == -5


def test_jvp_vjp_and_batched_report_nonfinite(checking):
    pr, z0 = fk(checkpoint_every=2)
    v = ri.direction(3, 70, 40, 1)
    with pytest.raises(rd.RDError) as e:
        rd.jvp(pr, dev(z0), dev(poisoned(v)))
    assert e.value.code == -5
    ck = torch.zeros(rd.checkpoint_count(pr) * 3 * pr.cells, dtype=torch.float64, device="cuda")
    rd.step(pr, dev(z0), ck)
    with pytest.raises(rd.RDError) as e:
        rd.vjp(pr, ck, dev(poisoned(v)))
    assert e.value.code == -5
    pr2, z2 = fk(nx=33, ny=20)
    with pytest.raises(rd.RDError) as e:
        rd.step_batched([pr, pr2], [dev(z0), dev(poisoned(z2))])
    assert e.value.code == -5 and "problem 1" in str(e.value)


def test_unchecked_call_lets_nan_through():
    pr, z0 = fk()
    z = dev(poisoned(z0))
    rd.step(pr, z)
    assert np.isnan(host(z)[0]).any()


def test_check_refused_inside_capture(checking):
    pr, z0 = fk()
    z = dev(z0)
    g = torch.cuda.CUDAGraph()
    stream = torch.cuda.Stream()
    stream.wait_stream(torch.cuda.current_stream())
    with pytest.raises(rd.RDError) as e:
        with torch.cuda.stream(stream):
            with torch.cuda.graph(g, stream=stream):
                rd.step(pr, z)
    assert e.value.code == -2
    torch.cuda.synchronize()
    assert all(np.array_equal(a, b) for a, b in zip(host(z), z0))
