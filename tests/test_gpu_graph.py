"""The step entry points enqueue kernels and copies only (no allocation, no
synchronisation, no memset), so a HIP graph can capture them: every replay
must equal the same call made eagerly, bit for bit.  Each test replays its
graph several times with other eager work and synchronisations in between,
and checks every replay."""
import numpy as np
import pytest
import torch

import paper_1309_1720_amd as rd
import rd_inputs as ri
from rdtest import dev, host, problems

pytestmark = pytest.mark.gpu

REPLAYS = 4


def eager_noise():
    """Unrelated eager device work between replays."""
    a = torch.rand(1 << 16, dtype=torch.float64, device="cuda")
    return float((a * 2.0 + 1.0).sum())


def test_batched_tangent_step_graph_replays():
    ws = ri.fk_batch_workloads(nsteps=3, sizes=(96, 130), per_size=3)
    params = ri.params_array("fk")
    probs = [rd.Problem.from_workload(w, params) for w in ws]
    z0 = [ri.fk_ic(w["nx"], w["ny"], w["seed"]) for w in ws]
    v0 = [ri.direction(3, w["nx"], w["ny"], w["direction_seed"]) for w in ws]
    # eager warm-up: the autotuner times its candidates outside the capture
    rd.step_batched(probs, [dev(z) for z in z0], [dev(v) for v in v0])
    torch.cuda.synchronize()

    fields, tans = [dev(z) for z in z0], [dev(v) for v in v0]
    ref_f, ref_t = [dev(z) for z in z0], [dev(v) for v in v0]
    g = torch.cuda.CUDAGraph()
    stream = torch.cuda.Stream()
    stream.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(stream):
        with torch.cuda.graph(g, stream=stream):
            rd.step_batched(probs, fields, tans)
    torch.cuda.current_stream().wait_stream(stream)
    # capturing ran nothing: the state is still the initial one
    assert all(np.array_equal(a, b) for a, b in zip(host(fields[0]), z0[0]))
    for rep in range(REPLAYS):
        g.replay()
        eager_noise()
        rd.step_batched(probs, ref_f, ref_t)
        torch.cuda.synchronize()
        for k in range(len(ws)):
            assert all(np.array_equal(a, b) for a, b in zip(host(fields[k]), host(ref_f[k]))), (rep, k)
            assert all(np.array_equal(a, b) for a, b in zip(host(tans[k]), host(ref_t[k]))), (rep, k)


@pytest.mark.parametrize("name,nsteps,every", [("barkley_128_euler", 37, 8), ("fk_1024_rk4", 5, 2)])
def test_single_grid_step_with_checkpoints_graph_replays(name, nsteps, every):
    w = ri.workload(name, nx=150, ny=97)
    _, pr = problems(w, nsteps=nsteps, checkpoint_every=every)
    z0 = ri.initial_condition(w)
    nv = len(z0)
    nck = rd.checkpoint_count(pr)
    rd.step(pr, dev(z0))  # warm-up (tuning)
    torch.cuda.synchronize()

    z, zr = dev(z0), dev(z0)
    ck = torch.zeros(nck * nv * w["nx"] * w["ny"], dtype=torch.float64, device="cuda")
    ckr = torch.zeros_like(ck)
    g = torch.cuda.CUDAGraph()
    stream = torch.cuda.Stream()
    stream.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(stream):
        with torch.cuda.graph(g, stream=stream):
            rd.step(pr, z, ck)
    torch.cuda.current_stream().wait_stream(stream)
    for rep in range(REPLAYS):
        g.replay()
        eager_noise()
        rd.step(pr, zr, ckr)
        torch.cuda.synchronize()
        assert all(np.array_equal(a, b) for a, b in zip(host(z), host(zr))), rep
        assert torch.equal(ck, ckr), rep


def test_captured_workspace_survives_larger_eager_calls_on_the_capture_stream():
    """Warm up on a side stream, capture on it, then run a larger problem
    eagerly on that same stream (which grows its cached workspace) and fill
    fresh allocations with other data; the graph's replays still equal eager
    runs: a captured call's workspace is its own and is never freed."""
    w = ri.workload("fk_1024_rk4", nx=150, ny=97)
    _, pr = problems(w, nsteps=4)
    _, big = problems(w, nsteps=2, nx=700, ny=500)
    z0 = ri.initial_condition(w)
    zb = ri.fk_ic(700, 500, 11)
    stream = torch.cuda.Stream()
    stream.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(stream):
        rd.step(pr, dev(z0))          # warm-up on the side stream (tuning, cached workspace)
        z = dev(z0)
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=stream):
            rd.step(pr, z)
        zr = dev(z0)
        for rep in range(REPLAYS):
            rd.step(big, dev(zb))      # larger workspace needed on this stream
            junk = torch.full((1 << 22,), float(rep + 1), dtype=torch.float64, device="cuda")
            rd.step(pr, zr)
            g.replay()
            del junk
            stream.synchronize()
            assert all(np.array_equal(a, b) for a, b in zip(host(z), host(zr))), rep
    torch.cuda.current_stream().wait_stream(stream)
