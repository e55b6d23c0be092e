"""Host-side parts of the time integrator (no device work): the kick and
drift factors against the FP64 oracle, and argument validation."""
import math

import pytest

import paper_2602_20787_amd as sc
from oracle import background as bg


@pytest.mark.parametrize("a0,a1,cos", [
    (0.02, 0.0212, dict(H0=0.944, Om=0.3, OL=0.7)),
    (0.5, 0.6, dict(H0=0.944, Om=0.3, OL=0.7)),
    (0.9, 1.0, dict(H0=1.3, Om=0.25, OL=0.7, Or=1e-4, Ok=0.0499)),
    (0.3, 0.33, dict(H0=1.0, Om=0.3, OL=0.7, w0=-0.9, wa=0.2)),
    (0.12, 0.1, dict(H0=0.944, Om=0.3, OL=0.7)),
])
def test_kdk_factors_match_oracle(a0, a1, cos):
    c = bg.Cosmology(**cos)
    p = sc.kdk_params(a0, a1, c.H0, c.Om, c.OL, c.Or, c.Ok, c.w0, c.wa)
    got = sc.steps_cyl_kdk_factors(p)
    ref = bg.kdk_factors(a0, a1, c)
    for g, r in zip(got, ref):
        assert g == pytest.approx(r, rel=1e-10)


@pytest.mark.parametrize("kw,code", [
    (dict(a_begin=0.0), sc.STEPS_EINVAL),
    (dict(a_end=-1.0), sc.STEPS_EINVAL),
    (dict(H0=0.0), sc.STEPS_EINVAL),
    (dict(Omega_m=math.nan), sc.STEPS_EINVAL),
    (dict(Omega_m=-2.0, Omega_L=0.1), sc.STEPS_EDOMAIN),
])
def test_kdk_factors_validation(kw, code):
    base = dict(a_begin=0.1, a_end=0.2, H0=1.0, Omega_m=0.3, Omega_L=0.7)
    base.update(kw)
    p = sc.kdk_params(**base)
    with pytest.raises(sc.StepsError) as e:
        sc.steps_cyl_kdk_factors(p)
    assert e.value.code == code


def test_kdk_step_rejects_bad_arguments():
    import ctypes
    p = sc.kdk_params(0.1, 0.2, 1.0, 0.3, 0.7, R_cyl=3.0, rho0=0.03)
    L = sc.lib()
    P = 8
    assert L.steps_cyl_kdk_step(None, P, P, P, 10, 1.0, ctypes.byref(p), P, None) == sc.STEPS_EINVAL
    assert L.steps_cyl_kdk_step(P, P, P, P, 0, 1.0, ctypes.byref(p), P, None) == sc.STEPS_EINVAL
    assert L.steps_cyl_kdk_step(P, P, P, P, 10, -1.0, ctypes.byref(p), P, None) == sc.STEPS_EINVAL
    bad = sc.kdk_params(0.1, 0.2, 1.0, 0.3, 0.7, R_cyl=-3.0, rho0=0.03)
    assert L.steps_cyl_kdk_step(P, P, P, P, 10, 1.0, ctypes.byref(bad), P, None) == sc.STEPS_EINVAL
    bad = sc.kdk_params(0.1, 0.2, 1.0, 0.3, 0.7, R_cyl=3.0, rho0=0.03, n_img=5000)
    assert L.steps_cyl_kdk_step(P, P, P, P, 10, 1.0, ctypes.byref(bad), P, None) == sc.STEPS_EINVAL
    assert L.steps_cyl_compensation(P, 10, -1.0, 8.5, 0.03, P, None) == sc.STEPS_EINVAL


# ---------------------------------------------------------------- tabulated history
def _lcdm_table(n):
    import numpy as np
    c = bg.Cosmology(H0=0.944, Om=0.3, OL=0.7)
    tt = np.linspace(bg.cosmic_time(0.05, c), bg.cosmic_time(0.5, c), n)
    aa = np.array([bg.lcdm_scale_factor(x, c) for x in tt])
    return tt, aa


@pytest.mark.parametrize("order", [1, 2, 3])
def test_history_factors_match_oracle(order):
    tt, aa = _lcdm_table(60)
    got = sc.steps_cyl_history_factors(tt, aa, order, 0.1, 0.13)
    ref = bg.history_factors(tt, aa, order, 0.1, 0.13)
    for g, r in zip(got, ref):
        assert g == pytest.approx(r, rel=1e-10)
    # reversed step
    got_r = sc.steps_cyl_history_factors(tt, aa, order, 0.13, 0.1)
    assert got_r[0] == pytest.approx(-got[2], rel=1e-9) and got_r[1] == pytest.approx(-got[1], rel=1e-9)


def test_history_factors_validation():
    import numpy as np
    tt, aa = _lcdm_table(10)
    with pytest.raises(sc.StepsError) as e:
        sc.steps_cyl_history_factors(tt, aa, 4, 0.1, 0.2)
    assert e.value.code == sc.STEPS_EINVAL
    with pytest.raises(sc.StepsError) as e:
        sc.steps_cyl_history_factors(tt, aa, 1, 0.01, 0.2)
    assert e.value.code == sc.STEPS_EDOMAIN
    bad = aa.copy()
    bad[4] = bad[3]
    with pytest.raises(sc.StepsError) as e:
        sc.steps_cyl_history_factors(tt, bad, 1, 0.1, 0.2)
    assert e.value.code == sc.STEPS_EINVAL
    with pytest.raises(sc.StepsError):
        sc.steps_cyl_history_factors(tt[:2], aa[:2], 3, 0.06, 0.07)


def test_explicit_factors_pass_through():
    # with factors given the background is not read (even nonsense values pass)
    p = sc.kdk_params(0.1, 0.2, -1.0, -1.0, -1.0, factors=(0.5, 0.25, 0.125))
    assert sc.steps_cyl_kdk_factors(p) == (0.5, 0.25, 0.125)
    bad = sc.kdk_params(0.1, 0.2, 1.0, 0.3, 0.7, factors=(0.5, float("nan"), 0.1))
    with pytest.raises(sc.StepsError) as e:
        sc.steps_cyl_kdk_factors(bad)
    assert e.value.code == sc.STEPS_EINVAL


def test_table_settings_are_checked():
    # a table handle is not dereferenced by the checks (host only)
    fake = 0x1000
    base = dict(a_begin=0.1, a_end=0.2, H0=1.0, Omega_m=0.3, Omega_L=0.7)
    with pytest.raises(sc.StepsError) as e:
        sc.steps_cyl_kdk_factors(sc.kdk_params(**base, table=fake, table_order=3))
    assert e.value.code == sc.STEPS_EINVAL and "table_order" in str(e.value)
    with pytest.raises(sc.StepsError) as e:
        sc.steps_cyl_kdk_factors(sc.kdk_params(**base, table=fake, net=fake))
    assert e.value.code == sc.STEPS_EINVAL
    # with a table n_img is not used
    sc.steps_cyl_kdk_factors(sc.kdk_params(**base, table=fake, table_order=1, n_img=-5))


def test_tree_settings_are_checked():
    fake = 0x1000
    base = dict(a_begin=0.1, a_end=0.2, H0=1.0, Omega_m=0.3, Omega_L=0.7)
    with pytest.raises(sc.StepsError) as e:
        sc.steps_cyl_kdk_factors(sc.kdk_params(**base, tree=fake))
    assert "needs a table" in str(e.value)
    with pytest.raises(sc.StepsError):
        sc.steps_cyl_kdk_factors(sc.kdk_params(**base, tree=fake, table=fake, theta=-1.0))
    with pytest.raises(sc.StepsError):
        sc.steps_cyl_kdk_factors(sc.kdk_params(**base, tree=fake, table=fake, tree_angle=float("inf")))
    sc.steps_cyl_kdk_factors(sc.kdk_params(**base, tree=fake, table=fake, theta=0.5))
