"""Pins of the display oracle (log compression, dynamic range, MIPs)."""
import numpy as np
import pytest

from oracle import display


def test_db_reference_and_floor():
    p = np.array([4.0, 0.4, 0.04, 4e-7, 0.0])
    d = display.display_db(p, 'power', 60.0)
    np.testing.assert_allclose(d, [0.0, -10.0, -20.0, -60.0, -60.0], atol=1e-12)
    # below the floor is shown at the floor, exactly
    assert display.display_db(np.array([1.0, 1e-9]), 'power', 60.0)[1] == -60.0


def test_amplitude_uses_twenty_log10():
    a = np.array([2.0, 0.2, 0.02 + 0.0j, 2j])
    d = display.display_db(a, 'iq', 75.0)
    np.testing.assert_allclose(d, [0.0, -20.0, -40.0, 0.0], atol=1e-12)
    # the phase of complex IQ does not matter, only |IQ|
    z = np.exp(1j * np.linspace(0, 6, 7)) * np.arange(1, 8)
    np.testing.assert_allclose(display.display_db(z, 'iq', 75.0), display.display_db(np.abs(z), 'iq', 75.0))


def test_scale_invariance_and_all_zero():
    rng = np.random.default_rng(0)
    p = rng.random(1000) ** 4
    np.testing.assert_allclose(display.display_db(p, 'power', 40.0), display.display_db(37.5 * p, 'power', 40.0),
                               atol=1e-12)
    np.testing.assert_array_equal(display.display_db(np.zeros(5), 'power', 60.0), -60.0)


def test_mip_against_loops_and_a_single_bright_voxel():
    rng = np.random.default_rng(1)
    nz, ny, nx = 5, 4, 3
    v = rng.random((nz, ny, nx))
    xy, xz, yz = (display.mip(v, p) for p in ('xy', 'xz', 'yz'))
    assert xy.shape == (ny, nx) and xz.shape == (nz, nx) and yz.shape == (nz, ny)
    for iy in range(ny):
        for ix in range(nx):
            assert xy[iy, ix] == max(v[iz, iy, ix] for iz in range(nz))
    for iz in range(nz):
        for ix in range(nx):
            assert xz[iz, ix] == max(v[iz, iy, ix] for iy in range(ny))
        for iy in range(ny):
            assert yz[iz, iy] == max(v[iz, iy, ix] for ix in range(nx))
    w = np.zeros((nz, ny, nx))
    w[3, 1, 2] = 5.0
    assert display.mip(w, 'xy')[1, 2] == 5.0 and display.mip(w, 'xz')[3, 2] == 5.0
    assert display.mip(w, 'yz')[3, 1] == 5.0 and display.mip(w, 'xy').sum() == 5.0


def test_log_display_commutes_with_mip():
    """dB is monotonic, so the dB of a MIP is the MIP of the dB volume (same reference)."""
    rng = np.random.default_rng(2)
    v = rng.random((6, 7, 8)) ** 3
    db = display.display_db(v, 'power', 30.0)
    for p in ('xy', 'xz', 'yz'):
        m = display.mip(v, p)
        np.testing.assert_allclose(display.mip(db, p), np.maximum(-30.0, 10 * np.log10(m / v.max())), atol=1e-12)


def test_unknown_kind_raises():
    with pytest.raises(ValueError):
        display.display_db(np.ones(3), 'bmode', 60.0)
