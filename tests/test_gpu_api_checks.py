"""GPU checks of the C ABI's contracts: caller-owned link words, the storage
scale chosen for a state near rest, and the calls that need a two-grid
layout refusing the buffer of an AA context."""
import numpy as np
import pytest
import torch

import lbm_inputs
from _helpers import dev, host

pytestmark = pytest.mark.gpu


def test_links_are_written_into_the_caller_buffer():
    """lbm_init writes the link words into the caller's buffer: bit 31 marks
    solid cells, bit q a fluid pull source x - c_q inside the lattice."""
    from paper_1803_04937_amd import Lattice, capi
    nx, ny, nz = 9, 7, 5
    solid = np.zeros((nz, ny, nx), np.uint8)
    solid[2, 3, 4] = 1
    lat = Lattice(nx, ny, nz, u=dev(np.zeros((3, nz, ny, nx))), solid=dev(solid, torch.uint8),
                  periodic=(1, 0, 1), dtype="f32")
    torch.cuda.synchronize()
    words = lat.links.cpu().numpy().view(np.uint32)[:nx * ny * nz].reshape(nz, ny, nx)
    c, _, _ = capi.lbm_velocity_set(19)
    assert words[2, 3, 4] >> 31 == 1
    assert np.count_nonzero(words >> 31) == 1
    # the cell at x + (1,0,0) pulls direction 1 from the solid cell: bit 1 clear
    assert (words[2, 3, 5] >> 1) & 1 == 0
    assert (words[2, 3, 6] >> 1) & 1 == 1
    # y walls: cells at y = 0 have no source below them in direction 3 (0,1,0)
    assert np.all((words[:, 0, :] >> 3) & 1 == 0)
    assert np.all((words[:, 1:, :][solid[:, :-1, :] == 0] >> 3) & 1 == 1)
    # after the words: the blocks with a fluid cell (here all of them, so the
    # kernels take every block and the list is not used)
    lat.close()


def test_active_block_list():
    """A mask whose solid cells fill whole 256-cell blocks: the list after
    the link words holds exactly the other blocks, ascending, and the step,
    AA step and adjoint over the list match the oracle."""
    import oracle
    from paper_1803_04937_amd import Lattice
    from _helpers import assert_adjoint_parity, assert_f64_parity
    nx, ny, nz = 64, 8, 6            # 4 rows per 256-cell block
    solid = np.zeros((nz, ny, nx), np.uint8)
    solid[1, 0:4, :] = 1             # rows 8-11: block 2 entirely solid
    solid[3, 4:8, :] = 1             # rows 28-31: block 7 entirely solid
    solid[4, 2, 10:20] = 1           # part of row 34 (block 8)
    cells = nx * ny * nz
    rng = np.random.default_rng(5)
    u0 = rng.uniform(-0.04, 0.04, (3, nz, ny, nx))
    cfg = oracle.Config(nx, ny, nz, periodic=(1, 1, 1), improved=1, trt=True, omega=1.6,
                        accel=(1e-4, 0, 0), solid=solid)
    for pattern in ("two_grid", "aa"):
        lat = Lattice(nx, ny, nz, u=dev(u0), solid=dev(solid, torch.uint8), equilibrium="improved",
                      collision="trt", omega=1.6, accel=(1e-4, 0, 0), dtype="f64",
                      pattern=pattern, adjoint_solid="skip")
        torch.cuda.synchronize()
        lst = lat.links.cpu().numpy().view(np.uint32)[cells:cells + cells // 256 - 2]
        np.testing.assert_array_equal(lst, [b for b in range(cells // 256) if b not in (2, 7)])
        lat.step(5)
        assert_f64_parity(host(lat.get_pdfs()), oracle.step(cfg, oracle.init(cfg, u0), 5),
                          f"active list {pattern}")
        lat.close()
    # adjoint over the list (solid cells left unwritten)
    lat = Lattice(nx, ny, nz, u=dev(u0), solid=dev(solid, torch.uint8), equilibrium="improved",
                  collision="trt", omega=1.6, accel=(1e-4, 0, 0), dtype="f64",
                  adjoint_solid="skip")
    f = host(lat.get_pdfs())
    lam = rng.standard_normal(f.shape)
    ln, lp = lat.new_adjoint(), lat.new_adjoint()
    lat.state_view(ln).copy_(dev(lam))
    grad = torch.zeros(4, dtype=torch.float64, device="cuda")
    lat.adjoint_step(lat.state, ln, lp, grad)
    want, gw = oracle.adjoint_step(cfg, f, lam)
    fl = solid == 0
    got = host(lat.state_view(lp))
    assert_adjoint_parity(got[:, fl], want[:, fl], "f64", "active list")
    np.testing.assert_allclose(host(grad), gw, rtol=1e-11, atol=1e-12 * np.abs(gw).max())
    lat.close()


def test_f16_near_rest_keeps_finite_totals():
    """FP16 storage from a state near rest (u ~ 1e-6 noise) driven by
    g = 2e-6: the scale is capped at 2^14, so s (f - w) stays representable
    as the flow develops and the totals stay finite and mass-conserving."""
    from paper_1803_04937_amd import Lattice
    n = 32
    u0 = lbm_inputs.perturbation((n, n, n), seed=3, amp=1e-6)
    lat = Lattice(n, n, n, u=dev(u0), periodic=(1, 0, 0), equilibrium="improved",
                  collision="trt", omega=1.95, accel=(2e-6, 0, 0), dtype="f16s")
    assert lat.scale == 2.0 ** 14
    m0 = lat.totals()[0]
    for _ in range(4):
        lat.step(500)
        tot = lat.totals()
        assert np.all(np.isfinite(tot)), tot
    assert abs(tot[0] - m0) / m0 < 1e-3
    assert tot[1] > 0.0     # the force has driven a flow along x
    lat.close()


def test_two_grid_calls_refuse_the_aa_buffer():
    from paper_1803_04937_amd import Lattice, capi
    n = 8
    lat = Lattice(n, n, n, u=dev(lbm_inputs.taylor_green(n, 0.02)), dtype="f32", pattern="aa")
    lam0, lam1 = lat.new_adjoint(), lat.new_adjoint()
    out = torch.zeros(4, dtype=torch.float64, device="cuda")
    with pytest.raises(capi.LBMError) as e:
        lat.objective(0, lat.state, out, lam0)
    assert e.value.status == capi.LBM_ESTATE
    with pytest.raises(capi.LBMError) as e:
        lat.adjoint_step(lat.state, lam0, lam1)
    assert e.value.status == capi.LBM_ESTATE
    # a two-grid state written by lbm_stream_collide is accepted
    a, b = lat.new_state(), lat.new_state()
    lat.set_pdfs(lat.get_pdfs())     # no-op round trip on the AA buffer
    lat2 = Lattice(n, n, n, u=dev(lbm_inputs.taylor_green(n, 0.02)), dtype="f32")
    lat2.copy_state(lat2.state, a)
    lat.stream_collide(a, b, 0)
    lat.objective(0, b, out, lam0)
    lat.adjoint_step(a, lam0, lam1)
    torch.cuda.synchronize()
    assert np.isfinite(out.cpu().numpy()).all()
    lat.close()
    lat2.close()
