"""Host replay of the shared reciprocals in the Bueno-Orovio rates (Eq. (5)
with the time constants of Bueno-Orovio et al. 2008).

The device code forms two reciprocals from one, 1/a = b (1/ab) and
1/b = a (1/ab), for (tau_v^-, tau_w^-) and (tau_so, tau_o), and writes
ds/dt = (s_inf - s)/tau_s with s_inf = 1/(1 + E) as
(1 - s (1 + E)) / ((1 + E) tau_s).  These checks replay those formulas in FP64
with numpy (each reciprocal correctly rounded, as the device's refined one is
to within an ulp) and compare them with the unshared forms evaluated in long
double, over voltages far beyond the physiological range: every product stays
finite (each holds at most one exponential, capped at e^600) and the results
agree to a few ulps.
"""
import numpy as np
import pytest

import rd_inputs as ri

EPS = np.finfo(np.float64).eps
CAP = 600.0  # the device's cap on the logistic exponent


def constants():
    q = ri.params_array("bocf").astype(np.float64)
    return dict(
        th_vm=q[4], th_o=q[5], th_w=q[3],
        tau_v1m=q[6], tau_v2m=q[7], tau_w1m=q[9], tau_w2m=q[10], k_wm=q[11], u_wm=q[12],
        tau_o1=q[15], tau_o2=q[16], tau_so1=q[17], tau_so2=q[18], k_so=q[19], u_so=q[20],
        tau_s1=q[21], tau_s2=q[22], k_s=q[23], u_s=q[24])


def heaviside_smooth(x, k):
    t = np.clip(k * x + 0.5, 0.0, 1.0)
    return (t * t) * (3.0 - 2.0 * t)


def capped_exp(k, u0, u):
    # E = e^(-2k(u - u0)): (1 + tanh(k(u - u0)))/2 = 1/(1 + E)
    return np.exp(np.minimum(-2.0 * k * u + 2.0 * k * u0, CAP))


VOLTAGES = np.concatenate([np.linspace(-50.0, 50.0, 20001), [-1e4, -700.0, -10.0, -6.0, -5.43, 1e4]])


@pytest.mark.parametrize("k", [ri.STEP_K, np.inf])
def test_tau_v_minus_and_tau_w_minus_share_one_reciprocal(k):
    c = constants()
    u = VOLTAGES
    h_vm = heaviside_smooth(u - c["th_vm"], k) if np.isfinite(k) else (u >= c["th_vm"]).astype(np.float64)
    E = capped_exp(c["k_wm"], c["u_wm"], u)
    d_wm = E * c["tau_w1m"] + c["tau_w2m"]
    t_vm = h_vm * (c["tau_v2m"] - c["tau_v1m"]) + c["tau_v1m"]
    R = 1.0 / (t_vm * d_wm)
    r_vm = R * d_wm
    r_wm = (1.0 + E) * (t_vm * R)
    assert np.isfinite(r_vm).all() and np.isfinite(r_wm).all()
    # unshared, in long double: 1/tau_v^- and (1 + E)/(tau_w1^- E + tau_w2^-)
    El = E.astype(np.longdouble)
    ref_vm = 1.0 / t_vm.astype(np.longdouble)
    ref_wm = (1.0 + El) / (El * c["tau_w1m"] + c["tau_w2m"])
    assert np.max(np.abs(r_vm - ref_vm) / ref_vm) <= 4 * EPS
    assert np.max(np.abs(r_wm - ref_wm) / ref_wm) <= 6 * EPS
    # the limits: 1/tau_w^- tends to 1/tau_w1^- far below rest and 1/tau_w2^- far above
    assert r_wm[u == -1e4][0] == pytest.approx(1.0 / c["tau_w1m"], rel=4 * EPS)
    assert r_wm[u == 1e4][0] == pytest.approx(1.0 / c["tau_w2m"], rel=4 * EPS)


@pytest.mark.parametrize("k", [ri.STEP_K, np.inf])
def test_tau_so_and_tau_o_share_one_reciprocal(k):
    c = constants()
    u = VOLTAGES
    h_o = heaviside_smooth(u - c["th_o"], k) if np.isfinite(k) else (u >= c["th_o"]).astype(np.float64)
    E = capped_exp(c["k_so"], c["u_so"], u)
    d_so = E * c["tau_so1"] + c["tau_so2"]
    t_o = h_o * (c["tau_o2"] - c["tau_o1"]) + c["tau_o1"]
    R = 1.0 / (t_o * d_so)
    r_so = (1.0 + E) * (t_o * R)
    r_o = R * d_so
    assert np.isfinite(r_so).all() and np.isfinite(r_o).all()
    El = E.astype(np.longdouble)
    ref_so = (1.0 + El) / (El * c["tau_so1"] + c["tau_so2"])
    ref_o = 1.0 / t_o.astype(np.longdouble)
    assert np.max(np.abs(r_so - ref_so) / ref_so) <= 6 * EPS
    assert np.max(np.abs(r_o - ref_o) / ref_o) <= 4 * EPS


def test_slow_gate_rate_with_one_reciprocal():
    """ds/dt = (s_inf - s)/tau_s.  Near s = s_inf the difference cancels in
    both forms, so the bound is absolute, on the scale (|s| + s_inf)/tau_s of
    the terms: a few ulps of it."""
    c = constants()
    rng = np.random.default_rng(7)
    u = np.repeat(VOLTAGES, 3)
    E = capped_exp(c["k_s"], c["u_s"], u)
    s_inf_ref = 1.0 / (1.0 + E.astype(np.longdouble))
    # s: uniform on [0, 1], and exactly at or one ulp beside its equilibrium
    s = rng.uniform(0.0, 1.0, u.size)
    s[1::3] = np.float64(s_inf_ref[1::3])
    s[2::3] = np.nextafter(np.float64(s_inf_ref[2::3]), 2.0)
    h_w = heaviside_smooth(u - c["th_w"], ri.STEP_K)
    tau_s = h_w * (c["tau_s2"] - c["tau_s1"]) + c["tau_s1"]
    one_e = 1.0 + E
    num = np.float64(1.0 - s.astype(np.longdouble) * one_e)  # one rounding, as the fused multiply-add
    f3 = num * (1.0 / (one_e * tau_s))
    assert np.isfinite(f3).all()
    ref = (s_inf_ref - s) / tau_s.astype(np.longdouble)
    scale = (np.abs(s) + s_inf_ref) / tau_s
    assert np.max(np.abs(f3 - ref) / scale) <= 6 * EPS
    # (within an ulp of s_inf the sign is not determined by either form: both
    # round s_inf, once or through 1 + E)


def test_device_source_uses_the_replayed_forms():
    import os
    src = open(os.path.join(os.path.dirname(__file__), "..", "paper_1309_1720_amd", "csrc", "rd_device.h")).read()
    for form in ("recip(t_vm * d_wm)", "t.r_vm = R * d_wm", "t.r_wm = (1.0 + E_wm) * (t_vm * R)",
                 "recip(t_o * d_so)", "r_so = (1.0 + E_so) * (t_o * R)", "r_o = R * d_so",
                 "mad(-s, one_e, T(1.0)) * recip(one_e * mad(t.h_w, m.dtau_s, T(m.tau_s1)))",
                 "kExpCap = 600.0"):
        assert form in src, form
