"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every entry point declared in include/lbm.h, encodes the same velocity set
as the oracle, and validates parameters before touching the GPU."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lbm.h")


@pytest.fixture(scope="module")
def capi():
    from paper_1803_04937_amd import capi as c
    return c


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lbm_[a-z_0-9]+)\s*\(", text)))


def test_every_declared_symbol_is_exported(capi):
    names = _declared()
    assert len(names) >= 20
    lib = ctypes.CDLL(capi.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(capi.EXPORTS) == names


@pytest.mark.parametrize("stencil", [19, 27])
def test_velocity_set_matches_oracle(capi, stencil):
    import oracle
    c, w, o = capi.lbm_velocity_set(stencil)
    oc, ow, oo = oracle.velocity_set(stencil)
    np.testing.assert_array_equal(np.array(c), oc)
    np.testing.assert_array_equal(np.array(w), ow)
    np.testing.assert_array_equal(np.array(o), oo)


def test_version(capi):
    assert "d3q19" in capi.lbm_version()


def test_layout_sizes(capi):
    """Plane-blocked buffers: nz planes of Q arrays of qstride elements,
    qstride = nx*ny rounded up to 64."""
    p = capi.make_params(256, 256, 256, dtype=capi.LBM_F32)
    qs = capi.lbm_qstride(p)
    assert qs == 256 * 256
    assert capi.lbm_state_bytes(p) == 256 * 19 * qs * 4
    assert capi.lbm_adjoint_bytes(p) == 256 * 19 * qs * 4
    p16 = capi.make_params(512, 512, 512, dtype=capi.LBM_F16_SHIFTED)
    assert capi.lbm_state_bytes(p16) == 512 * 19 * capi.lbm_qstride(p16) * 2
    p64 = capi.make_params(7, 5, 3, dtype=capi.LBM_F64)
    assert capi.lbm_qstride(p64) == 64
    assert capi.lbm_state_bytes(p64) == 3 * 19 * 64 * 8
    p27 = capi.make_params(37, 19, 15, dtype=capi.LBM_F32, stencil=27)
    assert capi.lbm_qstride(p27) == 704 and 704 % 64 == 0 and 704 >= 37 * 19
    assert capi.lbm_state_bytes(p27) == 15 * 27 * 704 * 4
    assert capi.lbm_adjoint_bytes(p27) == 15 * 27 * 704 * 4


BAD = [
    (dict(nx=0), "nx, ny, nz"),
    (dict(nx=2048, ny=2048, nz=512), "2^31"),
    (dict(omega=0.0), "omega"),
    (dict(omega=2.0), "omega"),
    (dict(omega=float("nan")), "omega"),
    (dict(collision=1, trt_magic=0.0), "trt_magic"),
    (dict(collision=1, trt_magic=-1.0), "trt_magic"),
    (dict(dtype=7), "dtype"),
    (dict(pattern=3), "pattern"),
    (dict(equilibrium=3), "equilibrium"),
    (dict(collision=5), "collision"),
    (dict(compressible=2), "compressible"),
    (dict(periodic=(1, 2, 1)), "periodic"),
    (dict(accel=(float("inf"), 0, 0)), "accel"),
    (dict(dtype=0, adjoint_dtype=1), "adjoint_dtype"),
    (dict(dtype=1, adjoint_dtype=0), "adjoint_dtype"),
    (dict(dtype=3, scale=3.0), "power of two"),
    (dict(stencil=15), "stencil"),
    (dict(collision=2, stencil=27), "MRT"),
    (dict(collision=2, mrt_omega3=0.0), "mrt_omega3"),
    (dict(collision=2, mrt_omega4=2.5), "mrt_omega4"),
    (dict(collision=4), "collision"),
    (dict(collision=3, stencil=27), "KBC"),
    (dict(open_x=2), "open_x"),
    (dict(open_x=1), "periodic[0]"),
    (dict(open_x=1, periodic=(0, 1, 1), pattern=1), "two-grid"),
    (dict(open_x=1, periodic=(0, 1, 1), compressible=1), "incompressible"),
    (dict(open_x=1, periodic=(0, 1, 1), rho_out=0.0), "rho_out"),
    (dict(rounding=2), "rounding"),
    (dict(cache_policy=3), "cache_policy"),
    (dict(adjoint_solid=2), "adjoint_solid"),
]


@pytest.mark.parametrize("kw,why", BAD)
def test_invalid_parameters_are_rejected(capi, kw, why):
    base = dict(nx=8, ny=8, nz=8)
    base.update(kw)
    p = capi.make_params(**base)
    rc, msg = capi.lbm_validate(p)
    assert rc == capi.LBM_EINVAL
    assert why in msg
    # lbm_init refuses the same parameters before any GPU call
    with pytest.raises(capi.LBMError) as e:
        capi.lbm_init(p, None, None, 1 << 20, 2 << 20, None, None, 3 << 20)
    assert e.value.status == capi.LBM_EINVAL
    assert why in str(e.value)


def test_init_argument_checks(capi):
    p = capi.make_params(8, 8, 8)
    for args, why in [((None, None, 0, 0, None, None, 1), "pdf0"),
                      ((None, None, 16, None, None, None, 1), "second"),
                      ((None, None, 16, 16, None, None, 1), "second"),
                      ((None, None, 16, 32, None, None, None), "u_init"),
                      ((64, None, 16, 32, None, None, 1), "link-word buffer")]:
        with pytest.raises(capi.LBMError) as e:
            capi.lbm_init(p, *args)
        assert why in str(e.value)
    paa = capi.make_params(8, 8, 8, pattern=capi.LBM_AA)
    with pytest.raises(capi.LBMError) as e:
        capi.lbm_init(paa, None, None, 16, 32, None, None, 1)
    assert "one buffer" in str(e.value)


def test_links_bytes(capi):
    p = capi.make_params(37, 19, 15)
    n = 37 * 19 * 15
    assert capi.lbm_links_bytes(p) == (n + (n + 255) // 256) * 4


def test_choose_scale_rule(capi):
    """Scale of the 16-bit formats: 2^floor(log2(1024 / maxdev)) clamped to
    [2^-10, 2^14], 2^14 at rest, monotone in maxdev, 1 for other dtypes; at
    the cap, s (f - w) stays inside FP16's normal range for |f - w| in
    [2^-28, 4)."""
    f16, bf16 = capi.LBM_F16_SHIFTED, capi.LBM_BF16_SHIFTED
    assert capi.lbm_choose_scale(f16, 0.0) == 2.0 ** 14
    assert capi.lbm_choose_scale(f16, 1e-6) == 2.0 ** 14     # near rest: capped
    assert capi.lbm_choose_scale(f16, 1e-30) == 2.0 ** 14
    assert capi.lbm_choose_scale(f16, 0.1) == 2.0 ** 13       # 1024 / 0.1 = 10240
    assert capi.lbm_choose_scale(f16, 1.0) == 2.0 ** 10
    assert capi.lbm_choose_scale(f16, 1e6) == 2.0 ** -10
    assert capi.lbm_choose_scale(bf16, 0.05) == 2.0 ** 14
    assert capi.lbm_choose_scale(capi.LBM_F32, 0.05) == 1.0
    devs = np.logspace(-12, 3, 400)
    s = [capi.lbm_choose_scale(f16, d) for d in devs]
    assert all(a >= b for a, b in zip(s, s[1:]))
    assert 4.0 * 2.0 ** 14 <= 65504 + 2.0 ** 14 and 2.0 ** -28 * 2.0 ** 14 == 2.0 ** -14
    for bad in (-1.0, float("nan"), float("inf")):
        with pytest.raises(capi.LBMError):
            capi.lbm_choose_scale(f16, bad)


def test_valid_parameters_pass(capi):
    for dt in range(5):
        p = capi.make_params(33, 17, 9, periodic=(1, 0, 0), dtype=dt, collision=capi.LBM_TRT,
                             omega=1.95, accel=(1e-6, 0, 0))
        assert capi.lbm_validate(p)[0] == capi.LBM_OK
