"""Pins of the oracle's non-isothermal network (the energy equation of
Sec. 4.2 at constant volume, synthetic thermodynamics): conservation of
internal energy and of elements by the right-hand side and along RKC
integrations, and the isothermal limit."""
import dataclasses

import numpy as np
import pytest

from paper_1611_02274_amd import inputs as I


def _parts(net, s):
    T, Y = s[0], s[1:]
    e = net.u0 + (net.cv0 + net.cv1 * T) * T
    cv = net.cv0 + 2.0 * net.cv1 * T
    return T, Y, e, cv


@pytest.mark.parametrize("n_sp", [9, 13])
def test_rhs_conserves_energy_and_elements(orc, n_sp):
    """d/dt sum_k Y_k e_k(T) = sum_k e_k dY_k/dt + c_v dT/dt = 0 and
    d/dt sum_k n_ke Y_k / W_k = 0 for every state."""
    net = I.thermal_network(n_sp)
    pb = orc.network_thermal(net)
    y0, g = I.thermal_inputs(net, 30, 77, (900.0, 2600.0))
    for i in range(30):
        s = y0[:, i]
        f = orc.rhs(pb, g[:, i], s)
        T, Y, e, cvk = _parts(net, s)
        cv = (Y * cvk).sum()
        terms = np.concatenate([e * f[1:], [cv * f[0]]])
        assert abs(terms.sum()) <= 1e-12 * np.abs(terms).sum()
        for el in range(3):
            v = net.comp[:, el] * f[1:] / net.W
            assert abs(v.sum()) <= 1e-12 * max(np.abs(v).sum(), 1e-300)


def test_integration_conserves_internal_energy(orc):
    net = I.thermal_network(9)
    pb = orc.network_thermal(net)
    y0, g = I.thermal_inputs(net, 12, 8008)
    y1, st, stats = orc.rkc_batch(pb, y0, g, 0.0, 1e-6, 1e-8, 1e-12)
    assert np.all(st == 0)
    assert np.abs(y1[0] - y0[0]).max() > 10.0            # temperature does change
    for i in range(12):
        T0, Y0, e0, _ = _parts(net, y0[:, i])
        T1, Y1, e1, _ = _parts(net, y1[:, i])
        u0, u1 = (Y0 * e0).sum(), (Y1 * e1).sum()
        scale = np.abs(Y0 * e0).sum()
        assert abs(u1 - u0) <= 1e-7 * scale
        assert abs(Y1.sum() - 1.0) <= 1e-11


def test_isothermal_limit(orc):
    """Equal specific heats independent of T and no formation energy: the
    energy equation keeps T exactly constant (mass conservation), and the
    species follow the isothermal network at that temperature."""
    base = I.thermal_network(13)
    cv = np.full(13, 1.2e7)
    net = dataclasses.replace(base, u0=np.zeros(13), cv0=cv, cv1=np.zeros(13))
    pb = orc.network_thermal(net)
    y0, g = I.thermal_inputs(net, 6, 99)
    f = orc.rhs(pb, g[:, 0], y0[:, 0])
    assert abs(f[0]) <= 1e-12 * np.abs(cv[0] * y0[0, 0] * f[1:]).sum() / cv[0]
    y1, st, _ = orc.rkc_batch(pb, y0, g, 0.0, 2e-7, 1e-10, 1e-14)
    assert np.all(st == 0)
    assert np.abs(y1[0] - y0[0]).max() <= 1e-9 * y0[0].max()
    iso = orc.network(net)
    gi = np.ascontiguousarray(np.stack([y0[0], g[0]]))
    yi, sti, _ = orc.rkc_batch(iso, np.ascontiguousarray(y0[1:]), gi, 0.0, 2e-7, 1e-10, 1e-14)
    assert np.abs(y1[1:] - yi).max() <= 1e-8
