"""The allocation-free moments entry point against lbm_moments, through the
C ABI: two calls in a row, the second on a smaller lattice (another dtype,
pattern and parity), each compared bit for bit with the context-based call;
and the size limit."""
import numpy as np
import pytest
import torch

import lbm_inputs
from _helpers import dev

pytestmark = pytest.mark.gpu


def _compare(lat):
    from paper_1803_04937_amd import capi
    n = lat.ncells
    rho_a = torch.empty(n, dtype=torch.float64, device="cuda")
    u_a = torch.empty(3 * n, dtype=torch.float64, device="cuda")
    sums_a = capi.lbm_moments(lat.ctx, rho_a, u_a, want_sums=True)
    rho_b = torch.full((n,), np.nan, dtype=torch.float64, device="cuda")
    u_b = torch.full((3 * n,), np.nan, dtype=torch.float64, device="cuda")
    sums_b = torch.full((4,), np.nan, dtype=torch.float64, device="cuda")
    capi.lbm_moments_noalloc(lat.params, lat.links, lat.state, lat.time, lat.scale, rho_b, u_b,
                             sums_b, lat.stream.cuda_stream)
    torch.cuda.synchronize()
    assert torch.equal(rho_a, rho_b)
    assert torch.equal(u_a, u_b)
    np.testing.assert_array_equal(np.array(sums_a), sums_b.cpu().numpy())
    return sums_a


def test_noalloc_moments_match_two_calls():
    from paper_1803_04937_amd import Lattice
    # first call: 96 x 80 x 64 with a mask, FP32 two-grid, force
    nx, ny, nz = 96, 80, 64
    solid = lbm_inputs.tube_mask(nx, ny, nz, r0=30.0, depth=0.4, centre=48.0, width=20.0)
    lat = Lattice(nx, ny, nz, u=dev(lbm_inputs.perturbation((nz, ny, nx), 1, 0.02)),
                  solid=dev(solid, torch.uint8), equilibrium="improved", collision="trt",
                  omega=1.7, accel=(1e-4, 0, 0), dtype="f32")
    lat.step(7)
    s1 = _compare(lat)
    assert np.isfinite(s1).all()
    lat.close()
    # second call, smaller: 40 x 24 x 20 periodic, FP16 AA after an odd step count
    n2 = (20, 24, 40)
    lat2 = Lattice(40, 24, 20, u=dev(lbm_inputs.perturbation(n2, 2, 0.03)), dtype="f16s",
                   pattern="aa", equilibrium="standard", collision="srt", omega=1.2)
    lat2.step(3)
    s2 = _compare(lat2)
    assert abs(s2[0] - 40 * 24 * 20) < 1e-6 * 40 * 24 * 20
    lat2.step(1)
    _compare(lat2)      # AA local layout again
    lat2.close()


def test_noalloc_rejects_too_many_cells():
    from paper_1803_04937_amd import capi
    p = capi.make_params(1024, 1024, 129, dtype=capi.LBM_F32)
    with pytest.raises(capi.LBMError) as e:
        capi.lbm_moments_noalloc(p, None, 1 << 20, 0, 1.0, None, None, None, None)
    assert e.value.status == capi.LBM_EINVAL
    assert "maximum" in str(e.value)
