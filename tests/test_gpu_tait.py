"""GPU parity with Tait water (Sec. 2.1; Case VI's water column, Table 2):
the library against the oracle on an air-water tube and on the
shock-helium-water set-up.  The Tait pressure uses pow(), whose last bit
may differ between the host's and the device's math libraries, so the bar is
the 1e-9 relative L1 error per conserved field (and the indicator field
exactly), not bit equality."""
import numpy as np
import pytest

import workloads as wl
from test_gpu_parity import assert_parity, run_both

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pk():
    import paper_1704_00519_amd as pk
    pk.load()
    return pk


@pytest.mark.parametrize("n,steps", [(400, 120), (333, 60)])
def test_air_water_tube(pk, n, steps):
    print("air-water tube", n, steps, flush=True)
    o, s = run_both(pk, wl.air_water_tube_1d(n=n), steps)
    assert_parity(o, s, label=f"air_water_{n}")
    assert s.diag()["n_updates"] == o.diag()["n_updates"]


@pytest.mark.parametrize("nx,ny,steps", [(128, 32, 40), (200, 56, 25)])
def test_shock_helium_water(pk, nx, ny, steps):
    print("shock-helium-water", nx, ny, steps, flush=True)
    o, s = run_both(pk, wl.shock_helium_water(nx=nx, ny=ny), steps)
    assert_parity(o, s, label=f"helium_water_{nx}x{ny}")
