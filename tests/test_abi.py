"""The C ABI library loads and exports every function include/ecpic.h
declares; configuration checks and state sizing run on the host (no GPU)."""
import ctypes as C
import os
import re

import pytest

from paper_2606_15035_amd import ecpic as E

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ecpic.h")


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(E.LIB_PATH):
        from paper_2606_15035_amd import build as B
        B.build()
    return E.lib()


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ecpic_[a-z_0-9]+)\s*\(", text)))


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert len(names) >= 15
    raw = C.CDLL(E.LIB_PATH)
    for n in names:
        assert hasattr(raw, n), n


def test_version_and_empty_error(lib):
    assert lib.ecpic_version().decode().startswith("ecpic-gfx950")
    assert isinstance(lib.ecpic_last_error(), bytes)


def good_cfg(**kw):
    args = dict(n=(32, 32, 32), L=(1.0, 1.0, 1.0), dt=0.1, r=2)
    args.update(kw)
    return E.make_config(**args)


def test_state_bytes_scale_with_particles(lib):
    s1, w1 = E.state_bytes(good_cfg(), 1000)
    s2, w2 = E.state_bytes(good_cfg(), 2000)
    per = (s2 - s1) / 1000
    # x, v, v^{n-1}, two iterates, the sort's second x, v, v^{n-1} (8 x 24 B)
    # plus id, second id and key (3 x 4 B), up to 256-byte alignment padding
    assert 204 <= per <= 210
    assert w2 >= w1 > 0


@pytest.mark.parametrize("bad", [
    dict(n=(32, 32, 30)),                 # not a power of two
    dict(n=(2, 32, 32)),                  # too small
    dict(r=4),                            # spline degree
    dict(r=0),
    dict(kappa=2.0),                      # sigma1 != kappa^2 sigma2
    dict(dt=0.0),
    dict(pmax=-1),
    dict(tol=-1.0),
    dict(precision=2),                    # no such precision
    dict(quad_points=17),                 # beyond the largest rule
    dict(quad_points=3),                  # split quadratic pieces need 4 points
    dict(r=3, quad_points=4),             # split cubic pieces need 5 points
    dict(split=False, precision=1),       # unsplit comparison path is FP64 only
    dict(scatter_chunk=1024),             # chunk lengths: 0 (automatic), 2048, 4096
    dict(r=3, scatter_chunk=4096),        # cubic stencils take 2048
])
def test_invalid_configurations_are_rejected(lib, bad):
    with pytest.raises(E.EcpicError) as ei:
        E.state_bytes(good_cfg(**bad), 10)
    assert ei.value.status == E.EINVAL
    assert len(lib.ecpic_last_error()) > 0


@pytest.mark.parametrize("count", [-1, 2 ** 31])
def test_particle_count_outside_the_32_bit_range_is_rejected(lib, count):
    with pytest.raises(E.EcpicError) as ei:
        E.state_bytes(good_cfg(), count)
    assert ei.value.status == E.EINVAL
    E.state_bytes(good_cfg(), 2 ** 31 - 1)  # the largest count is accepted


def test_mixed_precision_state_is_smaller(lib):
    s64, _ = E.state_bytes(good_cfg(), 100000)
    smx, _ = E.state_bytes(good_cfg(precision=E.MIXED), 100000)
    # per particle: x, v, v^{n-1} and their sort copies shrink from 144 B
    # (FP64) to 80 B (int32 cell, FP32 offset, FP32 v, FP32 v^{n-1})
    assert 60 <= (s64 - smx) / 100000 <= 68


@pytest.mark.parametrize("m", [-1, 5])
def test_anderson_depth_range(lib, m):
    with pytest.raises(E.EcpicError) as ei:
        E.state_bytes(good_cfg(anderson=m), 10)
    assert ei.value.status == E.EINVAL


def test_anderson_history_is_state(lib):
    # depth m keeps the iterates and images of m more passes: 2 m x 24 B per particle
    s0, _ = E.state_bytes(good_cfg(), 100000)
    for m in (1, 2, 4):
        s, _ = E.state_bytes(good_cfg(anderson=m), 100000)
        assert 48 * m <= (s - s0) / 100000 <= 48 * m + 1


@pytest.mark.parametrize("scale", [-1.0, 2.0 ** 53])
def test_fixed_point_scale_range(lib, scale):
    with pytest.raises(E.EcpicError):
        E.state_bytes(good_cfg(precision=E.MIXED, fixed_point_scale=scale), 10)


@pytest.mark.parametrize("ok", [dict(split=False), dict(split=False, quad_points=16),
                                dict(split=False, quad_points=1), dict(quad_points=16)])
def test_unsplit_and_larger_rules_accepted(lib, ok):
    E.state_bytes(good_cfg(**ok), 10)


def test_maxwell_scaling_accepted_when_consistent(lib):
    E.state_bytes(good_cfg(kappa=2.0, sigma1=4.0, sigma2=1.0), 10)


def test_negative_particle_count_rejected(lib):
    with pytest.raises(E.EcpicError):
        E.state_bytes(good_cfg(), -1)


def test_create_rejects_small_or_misaligned_buffers(lib):
    cfg = good_cfg()
    s, w = E.state_bytes(cfg, 100)
    h = C.c_void_p()
    # buffers too small (addresses are never dereferenced: the size check comes first)
    st = lib.ecpic_create(C.byref(cfg), 100, C.c_void_p(4096), 16, C.c_void_p(8192), 16, None,
                          C.byref(h))
    assert st == E.ENOMEM
    st = lib.ecpic_create(C.byref(cfg), 100, C.c_void_p(4096 + 8), s, C.c_void_p(8192), w, None,
                          C.byref(h))
    assert st == E.EINVAL
    st = lib.ecpic_create(C.byref(cfg), 100, None, s, None, w, None, C.byref(h))
    assert st == E.EINVAL
