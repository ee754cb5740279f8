"""Host-only checks of the C ABI: the library loads, exports every function
include/rd.h declares, and rejects bad arguments before touching a device."""
import ctypes as C
import math
import os
import re

import pytest

import paper_1309_1720_amd as rd
from paper_1309_1720_amd import _binding as B
import rd_inputs as ri

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "rd.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\**\s*(rd_\w+)\s*\(", text, flags=re.M)))


def test_library_exports_every_declared_function():
    names = declared_functions()
    assert {"rd_step", "rd_jvp", "rd_vjp", "rd_step_batched"} <= set(names)
    L = rd.lib()
    for n in names:
        assert hasattr(L, n), n


def test_abi_version_and_counts():
    L = rd.lib()
    assert L.rd_abi_version() == B.ABI_VERSION
    for m, n in ri.N_FIELDS.items():
        assert rd.n_fields(m) == n
        assert rd.n_params(m) == len(ri.PARAM_NAMES[m])
    assert L.rd_n_fields(7) == -1


def base_problem(**kw):
    w = ri.workload("fk_1024_rk4", nx=64, ny=48, nsteps=3)
    p = rd.Problem.from_workload(w, ri.params_array("fk"))
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def call_step(p, fields=True, ws=True, ws_bytes=None):
    cp, buf = p.to_c()
    nv = p.nfields
    fake = (C.c_void_p * nv)(*[0x10000 * (i + 1) for i in range(nv)]) if fields else None
    need = C.c_size_t(0)
    B.lib().rd_workspace_bytes(C.byref(cp), 0, C.byref(need))
    nbytes = need.value if ws_bytes is None else ws_bytes
    rc = B.lib().rd_step(C.byref(cp), fake, None, 0x100000 if ws else None, nbytes, None)
    return rc, B.lib().rd_last_error().decode()


@pytest.mark.parametrize("field,value,code", [
    ("nx", 0, -1), ("ny", -3, -1), ("dx", 0.0, -1), ("dt", -0.1, -1), ("dt", math.nan, -1),
    ("nsteps", -1, -1), ("step_k", 0.0, -1), ("D_par", math.inf, -1),
])
def test_invalid_scalars_rejected(field, value, code):
    rc, msg = call_step(base_problem(**{field: value}))
    assert rc == code and msg


def test_invalid_enums_and_params_rejected():
    for kw in ({"params": (1.0, 2.0)}, {"params": tuple([math.nan] * 13)}):
        rc, msg = call_step(base_problem(**kw))
        assert rc == -1 and msg
    p = base_problem()
    cp, buf = p.to_c()
    for fld, bad in (("model", 9), ("scheme", 3), ("stencil", 6), ("bc", 2), ("abi_version", 99)):
        q = B._CProblem.from_buffer_copy(cp)
        setattr(q, fld, bad)
        rc = B.lib().rd_step(C.byref(q), (C.c_void_p * 3)(1 << 16, 2 << 16, 3 << 16), None, 1 << 20, 1 << 30, None)
        assert rc == -1, fld


def test_null_and_small_workspace_rejected():
    assert call_step(base_problem(), fields=False)[0] == -1
    assert call_step(base_problem(), ws=False)[0] == -3
    assert call_step(base_problem(), ws_bytes=16)[0] == -3
    assert B.lib().rd_step(None, None, None, None, 0, None) == -1


def test_grid_too_large_rejected():
    rc, msg = call_step(base_problem(nx=1 << 16, ny=1 << 15))
    assert rc == -1 and "2^31" in msg


def test_workspace_and_checkpoint_queries():
    p = base_problem(nsteps=130, checkpoint_every=64)
    assert rd.checkpoint_count(p) == 3
    assert rd.workspace_bytes(p, "step") >= 3 * 64 * 48 * 8
    p.checkpoint_every = 0
    assert rd.checkpoint_count(p) == 0


def test_zero_steps_is_a_noop_without_device():
    rc, _ = call_step(base_problem(nsteps=0), ws=False)
    assert rc == 0


def test_steps_per_launch_knob():
    L = B.lib()
    for bad in (3, 5, 16):
        assert L.rd_set_steps_per_launch(bad) == -1
        assert "steps per launch" in L.rd_last_error().decode()
    try:
        w = ri.workload("barkley_128_euler")
        pb = rd.Problem.from_workload(w, ri.params_array("barkley"))
        pf = base_problem()
        rd.set_steps_per_launch(8)
        assert rd.get_steps_per_launch(pb) == 8       # Euler chains up to 8 steps
        pb.scheme = "rk4"
        assert rd.get_steps_per_launch(pb) == 2       # RK4: 2 steps (8 stages)
        assert rd.get_steps_per_launch(pf) == 1       # gated models: one step
        rd.set_steps_per_launch(None)
        assert rd.get_steps_per_launch(pb) == 1       # untuned start
    finally:
        rd.set_steps_per_launch(None)


def test_fhn_model_tables_and_negative_delta_rejected():
    assert rd.n_fields("fhn") == 2 and rd.n_params("fhn") == 4
    w = ri.workload("fhn_256_rk4", nx=32, ny=24)
    p = rd.Problem.from_workload(w, ri.params_array("fhn", {"delta": -0.5}))
    cp, _buf = p.to_c()
    out = C.c_size_t(0)
    assert B.lib().rd_workspace_bytes(C.byref(cp), 0, C.byref(out)) == -1
    assert "delta" in B.lib().rd_last_error().decode()


def test_krylov_vector_calls_validate_before_launch():
    L = B.lib()
    need = C.c_size_t(0)
    assert L.rd_vec_gram_workspace_bytes(0, C.byref(need)) == -1
    assert L.rd_vec_gram_workspace_bytes(65, C.byref(need)) == -1
    assert L.rd_vec_gram_workspace_bytes(3, C.byref(need)) == 0 and need.value >= 3 * 8
    xs = (C.c_void_p * 3)(0x1000, 0x2000, 0x3000)
    # too small a workspace, NULL output, bad sizes: rejected on the host
    assert L.rd_vec_gram(xs, 3, 0x4000, 10, 0x5000, 0x6000, 8, None) == -3
    assert L.rd_vec_gram(xs, 3, 0x4000, 10, None, 0x6000, need.value, None) == -1
    assert L.rd_vec_gram(xs, 3, 0x4000, 0, 0x5000, 0x6000, need.value, None) == -1
    coef = (C.c_double * 3)(1.0, 2.0, 3.0)
    assert L.rd_vec_lincomb(0x7000, 1.0, xs, coef, -1, 10, None) == -1
    assert L.rd_vec_lincomb(0x7000, 1.0, xs, coef, 65, 10, None) == -1
    assert L.rd_vec_lincomb(None, 1.0, xs, coef, 3, 10, None) == -1
    assert L.rd_vec_lincomb(0x7001, 1.0, xs, coef, 3, 10, None) == -1


def test_gate_schemes_need_gated_models():
    w = ri.workload("barkley_128_euler", scheme="rush_larsen")
    pb = rd.Problem.from_workload(w, ri.params_array("barkley"))
    cp, _b = pb.to_c()
    out = C.c_size_t(0)
    assert B.lib().rd_workspace_bytes(C.byref(cp), 0, C.byref(out)) == -2
    assert "gated model" in B.lib().rd_last_error().decode()
    # rd_vjp refuses a gate scheme on a model without gates before anything
    # is enqueued
    pb.checkpoint_every = 2
    cpb, _b2 = pb.to_c()
    fake = (C.c_void_p * 2)(0x10000, 0x20000)
    rc = B.lib().rd_vjp(C.byref(cpb), 0x40000, fake, 0x100000, 1 << 30, None)
    assert rc == -2 and "gated model" in B.lib().rd_last_error().decode()


def test_3d_problems_validated_before_any_device_work():
    # nz must be 1 for the 2-D stencils and >= 1 for the 3-D ones
    rc, msg = call_step(base_problem(nz=2))
    assert rc == -1 and "nz" in msg
    rc, msg = call_step(base_problem(stencil="lap19", nz=0))
    assert rc == -1 and "nz" in msg
    rc, msg = call_step(base_problem(stencil="lap27", nx=1 << 14, ny=1 << 14, nz=1 << 12))
    assert rc == -1 and "2^40" in msg
    # workspace: the ping-pong state plus NS - 1 stored rates, NV (or 2 NV) fields each
    p = base_problem(stencil="lap27", nx=30, ny=20, nz=10)
    fb = -(-30 * 20 * 10 * 8 // 256) * 256
    assert rd.workspace_bytes(p, "step") == 4 * 3 * fb
    assert rd.workspace_bytes(p, "jvp") == 4 * 6 * fb
    p.scheme = "heun"
    assert rd.workspace_bytes(p, "step") == 2 * 3 * fb
    # adjoint: (C - 1) states, NS - 1 rates, two Ybar buffers, zbar and the cotangent partner
    p.checkpoint_every = 5
    assert rd.workspace_bytes(p, "vjp") == 3 * (4 + 1 + 4) * fb
    cp, _b = p.to_c()
    v, r = C.c_int32(), C.c_int32()
    assert B.lib().rd_get_plan(C.byref(cp), 0, C.byref(v), C.byref(r)) == -2
    bb = C.c_size_t()
    assert B.lib().rd_step_batched_workspace_bytes(C.byref(cp), 1, 0, C.byref(bb)) == 0
    assert bb.value == rd.workspace_bytes(p, "step")   # one instance: its own stage workspace
    # rejected before any launch: no checkpoint spacing, no planes
    fake = (C.c_void_p * 3)(1 << 16, 2 << 16, 3 << 16)
    for kw in ({"checkpoint_every": 0}, {"nz": 0}):
        q = base_problem(stencil="lap27", nx=30, ny=20, nz=10, checkpoint_every=5)
        for k, val in kw.items():
            setattr(q, k, val)
        cq, _bq = q.to_c()
        assert B.lib().rd_vjp(C.byref(cq), C.c_void_p(1 << 20), fake, C.c_void_p(1 << 24), 1 << 30, None) in (-1, -2)


def test_check_finite_knob_adds_workspace():
    p = base_problem(nsteps=7, checkpoint_every=3)
    base = {op: rd.workspace_bytes(p, op) for op in ("step", "jvp", "vjp")}
    bb = C.c_size_t()
    cp, _b = p.to_c()
    assert B.lib().rd_step_batched_workspace_bytes(C.byref(cp), 1, 1, C.byref(bb)) == 0
    rd.set_check_finite(True)
    try:
        for op, n in base.items():
            assert rd.workspace_bytes(p, op) == n + 256, op
        b2 = C.c_size_t()
        assert B.lib().rd_step_batched_workspace_bytes(C.byref(cp), 1, 1, C.byref(b2)) == 0
        assert b2.value == bb.value + 256
    finally:
        rd.set_check_finite(False)
    assert rd.workspace_bytes(p, "step") == base["step"]
    assert B.STATUS[-5] == "RD_ENONFINITE"


def test_workspace_bytes_takes_a_batch():
    """rd_workspace_bytes(p, RD_OP_BATCHED[_JVP], out) sizes rd_step_batched for
    the batch p[0 .. nbatch-1], nbatch read from *out; the separate
    rd_step_batched_workspace_bytes is the same query."""
    sizes = [(64, 48), (33, 17), (100, 7)]
    probs = [base_problem(nx=nx, ny=ny) for nx, ny in sizes]
    cps, bufs = zip(*[p.to_c() for p in probs])
    arr = (B._CProblem * len(probs))(*cps)
    L = B.lib()
    for op, tangents in ((3, 0), (4, 1)):
        out = C.c_size_t(len(probs))
        assert L.rd_workspace_bytes(arr, op, C.byref(out)) == 0, L.rd_last_error()
        alias = C.c_size_t(0)
        assert L.rd_step_batched_workspace_bytes(arr, len(probs), tangents, C.byref(alias)) == 0
        assert out.value == alias.value
        # descriptor table (256-byte aligned) + one partner array per instance array
        fields = sum((1 + tangents) * 3 * (-(-nx * ny * 8 // 256) * 256) for nx, ny in sizes)
        assert fields < out.value <= fields + 256 * len(probs) + 4096
        # a prefix of the batch needs less
        out1 = C.c_size_t(1)
        assert L.rd_workspace_bytes(arr, op, C.byref(out1)) == 0
        assert out1.value < out.value
    assert rd.workspace_bytes(probs, "batched") < rd.workspace_bytes(probs, "batched_jvp")
    # nbatch out of range on entry, or an invalid member: refused, *out untouched
    for n in (0, 65537):
        out = C.c_size_t(n)
        assert L.rd_workspace_bytes(arr, 3, C.byref(out)) == -1
        assert out.value == n
    bad = base_problem(nx=0)
    cb, _bb = bad.to_c()
    arr2 = (B._CProblem * 2)(cps[0], cb)
    out = C.c_size_t(2)
    assert L.rd_workspace_bytes(arr2, 3, C.byref(out)) == -1
    assert "problem 1" in L.rd_last_error().decode()
    assert L.rd_workspace_bytes(arr, 3, None) == -1
    assert L.rd_workspace_bytes(arr, 9, C.byref(C.c_size_t(1))) == -1
    del bufs
