"""The oracle's terrain friction against the closed form of a block sliding on
an inclined plane (the sliding-box benchmark of the paper's examples: slope
angles 14, 20, 25, 30 degrees, mu = tan 15 degrees, elastic block).

A rigid block released at rest on a plane of slope theta with Coulomb
coefficient mu moves down the slope by d(t) = g (sin theta - mu cos theta) t^2 / 2
when tan theta > mu, and stays put otherwise.  The simulated block is elastic
(E = 5e5 Pa): after its release it settles onto the plane and shears under
its weight, a transient of a few millimetres, which shrinks in proportion to
1/E (at 14 degrees the displacement after 0.3 s is 14.0, 3.3 and 0.31 mm for
E = 5e4, 5e5 and 5e6 Pa, and the block comes to rest: the node-level Coulomb
condition holds it).  Pins, on the centre of mass's downslope displacement:

  20 degrees, t = 0.3 s: d within 12 % of the closed form 39.4 mm (measured
  +8.3 %, the settling transient; a 10 % error in mu or a dropped cos theta
  moves d by 17-28 %), and the acceleration fitted over [0.05, 0.3] s within
  2 % (measured 0.2 %);
  14 degrees, t = 0.3 s: |d| <= 5 mm (the closed form is 0; at 20 degrees the
  block has moved 43 mm by then; measured 3.3 mm, the settling) and the
  velocity over the last 0.05 s below 1 cm/s (measured 0.09 cm/s: at rest).
"""
import numpy as np
import pytest

from oracle import mpm as om
from paper_2605_28525_amd import workloads as wl

T_FIT0, T_END = 0.05, 0.3
G = 9.81


def closed_form_acceleration(theta_deg: float, mu: float = wl.SLIDE_MU) -> float:
    th = np.deg2rad(theta_deg)
    return max(0.0, G * (np.sin(th) - mu * np.cos(th)))


def fit_acceleration(t, d, t0=T_FIT0):
    t, d = np.asarray(t), np.asarray(d)
    sel = t >= t0 - 1e-12
    return 2.0 * np.polyfit(t[sel], d[sel], 2)[0]


def sample_every(w) -> int:
    return max(1, int(round(0.01 / w.dt)))


def oracle_curve(theta_deg: float, t_end: float = T_END):
    """(t, downslope displacement of the centre of mass) every ~0.01 s."""
    w = wl.sliding_block(theta_deg)
    p = om.Params.from_workload(w)
    st = om.state_from_soa(w.state(), 3)
    t_hat = w.meta["downslope"]
    c0 = st["x"].mean(axis=0)
    every, n = sample_every(w), int(round(t_end / w.dt))
    ts, ds = [], []
    for k in range(1, n + 1):
        st = om.step(st, p)
        if k % every == 0:
            ts.append(k * w.dt)
            ds.append(float((st["x"].mean(axis=0) - c0) @ t_hat))
    return np.array(ts), np.array(ds)


def test_closed_form_acceleration_values():
    # tan 14 < mu = tan 15 < tan 20: stick at 14, slide at the others
    assert closed_form_acceleration(14.0) == 0.0
    assert np.isclose(closed_form_acceleration(15.0), 0.0, atol=1e-12)
    assert np.isclose(closed_form_acceleration(20.0), 0.8846, atol=1e-3)
    assert np.isclose(closed_form_acceleration(30.0), 2.6286, atol=1e-3)
    assert closed_form_displacement(14.0, 0.3) == 0.0
    assert np.isclose(closed_form_displacement(20.0, 0.3), 0.5 * 0.8852 * 0.09, rtol=1e-3)


def test_fit_recovers_a_quadratic():
    t = np.linspace(0.0, 0.15, 16)
    d = 0.003 + 0.04 * t + 0.5 * 1.7 * t * t
    assert np.isclose(fit_acceleration(t, d), 1.7, rtol=1e-9)


def test_sliding_block_workload_geometry():
    w = wl.sliding_block(25.0)
    th = np.deg2rad(25.0)
    x = w.x.astype(np.float64)
    # every particle lies above the plane, within the block's 0.1 m thickness
    dist = (x[2] - (0.6 - x[0] * np.tan(th))) * np.cos(th)
    assert dist.min() > 0 and dist.max() < 0.1
    # the heightmap is the plane at the nodes
    X = np.arange(w.cells[0] + 1) * w.dx
    assert np.allclose(w.heightmap[:, 0], 0.6 - X * np.tan(th), atol=1e-6)
    assert w.n == 10 * 5 * 5 * 8


def closed_form_displacement(theta_deg: float, t, mu: float = wl.SLIDE_MU):
    return 0.5 * closed_form_acceleration(theta_deg, mu) * np.asarray(t) ** 2


def late_velocity(t, d, span=0.05):
    """Slope of the displacement over the last `span` seconds."""
    t, d = np.asarray(t), np.asarray(d)
    sel = t >= t[-1] - span - 1e-12
    return np.polyfit(t[sel], d[sel], 1)[0]


# (relative displacement bound, acceleration bound) where the block slides;
# (displacement bound m, velocity bound m/s) where it sticks
SLIDE_BOUNDS = (0.12, 0.02)
STICK_BOUNDS = (5e-3, 1e-2)
T_STICK = 0.3


def check_sliding_curve(theta, t, d):
    """The pins above, shared by the oracle's and the GPU's curves."""
    a_ref = closed_form_acceleration(theta)
    if a_ref > 0:
        a = fit_acceleration(t, d)
        d_ref = float(closed_form_displacement(theta, t[-1]))
        print(f"theta {theta}: d({t[-1]:.3f}) {d[-1] * 1e3:.2f} mm, closed form {d_ref * 1e3:.2f} mm; "
              f"a {a:.4f}, closed form {a_ref:.4f}", flush=True)
        assert abs(d[-1] - d_ref) <= SLIDE_BOUNDS[0] * d_ref, (d[-1], d_ref)
        assert abs(a - a_ref) <= SLIDE_BOUNDS[1] * a_ref, (a, a_ref)
    else:
        v = late_velocity(t, d)
        print(f"theta {theta}: d({t[-1]:.3f}) {d[-1] * 1e3:.2f} mm, late velocity {v * 1e2:.3f} cm/s", flush=True)
        assert abs(d[-1]) <= STICK_BOUNDS[0], d[-1]
        assert abs(v) <= STICK_BOUNDS[1], v


@pytest.mark.parametrize("theta,t_end", [(20.0, T_END), (14.0, T_STICK)])
def test_oracle_sliding_displacement(theta, t_end):
    t, d = oracle_curve(theta, t_end)
    check_sliding_curve(theta, t, d)
