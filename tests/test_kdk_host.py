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
