"""C-ABI checks that need no GPU: the library loads, exports every symbol
include/lbm.h declares, validates configurations, and reports the documented
direction order."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import oracle as O
from paper_1710_02065_amd import lbm

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                      "include", "lbm.h")


def declared_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(lbm_[a-z_0-9]+)\s*\(", txt)))


def test_library_exports_every_declared_function():
    names = declared_functions()
    assert len(names) >= 18
    L = lbm.lib()
    for n in names:
        assert hasattr(L, n), n
    assert sorted(lbm.EXPORTS) == names


def test_config_struct_size_matches_binding():
    cfg = lbm.lbm_config_init()
    assert cfg.struct_size == C.sizeof(lbm.lbm_config)


@pytest.mark.parametrize("q", [9, 19, 27])
def test_direction_order_matches_oracle(q):
    xi, w = lbm.lbm_lattice_table(q)
    oxi, ow, _ = O.lattice(q)
    np.testing.assert_array_equal(xi, oxi)
    np.testing.assert_allclose(w, ow, rtol=0, atol=1e-17)


def required(**kw):
    return lbm.lbm_required_bytes(lbm.make_config(**kw))


def test_required_bytes_counts_both_buffers():
    n = required(lattice=19, shape=(64, 64, 64), storage="f32")
    pop = 64 ** 3 * 4 * 19 * 2
    assert pop <= n < pop * 1.01 + (1 << 20)
    assert required(lattice=19, shape=(64, 64, 64), storage="f16s") < n * 0.6
    assert required(lattice=9, shape=(128, 128, 1), storage="f64") >= 128 * 128 * 9 * 8 * 2


@pytest.mark.parametrize("bad,msg", [
    (dict(tau=0.5), "tau"),
    (dict(tau=0.6, chi_max=2.4), "chi_max"),
    (dict(ma=0.7), "Ma"),
    (dict(lattice=15), "lattice"),
    (dict(storage=7), "storage"),
    (dict(lattice=9, shape=(8, 8, 2)), "nz"),
    (dict(face_bc=(0, 1, 0, 0, 0, 0)), "periodic"),
    (dict(shape=(2048, 2048, 1024)), "2^31"),
    (dict(sponge_width=(100, 0, 0, 0, 0, 0)), "sponge"),
])
def test_invalid_configurations_rejected(bad, msg):
    kw = dict(lattice=19, shape=(64, 64, 64))
    kw.update(bad)
    assert required(**kw) == 0
    assert msg.lower() in lbm.lbm_last_error().lower()


def test_high_mach_flag():
    assert required(ma=0.7, flags=lbm.LBM_ALLOW_HIGH_MA) > 0


def test_create_without_device_reports_error():
    """On a machine without a GPU, create fails cleanly (no crash)."""
    try:
        import torch
        if torch.cuda.is_available():
            pytest.skip("a GPU is present")
    except ImportError:
        pass
    with pytest.raises(lbm.LbmError) as e:
        lbm.lbm_create(lbm.make_config())
    assert e.value.code in (lbm.LBM_EDEVICE, lbm.LBM_EINVAL)


@pytest.mark.parametrize("bad,msg", [
    (dict(refine_lo=(2, 10, 10), refine_hi=(20, 30, 30)), "must lie"),
    (dict(refine_lo=(10, 10, 10), refine_hi=(12, 30, 30)), "< 4"),
    (dict(refine_lo=(10, 10, 10), refine_hi=(60, 30, 30)), "must lie"),
    (dict(refine_lo=(10, 10, 10), refine_hi=(30, 30, 30), sponge_width=(12, 0, 0, 0, 0, 0)),
     "absorbing"),
    (dict(lattice=9, shape=(64, 64, 1), refine_lo=(10, 10, 1), refine_hi=(30, 30, 1)), "z range"),
])
def test_invalid_refinement_rejected(bad, msg):
    kw = dict(lattice=19, shape=(64, 64, 64))
    kw.update(bad)
    assert required(**kw) == 0
    assert msg.lower() in lbm.lbm_last_error().lower()


def test_refined_required_bytes_counts_fine_level():
    base = required(lattice=19, shape=(64, 64, 64), storage="f32")
    ref = required(lattice=19, shape=(64, 64, 64), storage="f32", refine_lo=(10, 10, 10),
                   refine_hi=(30, 30, 30))
    fine = 41 ** 3 * 19 * 4 * 2
    assert ref >= base + fine


def test_full_order_needs_d2q9_or_d3q27():
    assert required(lattice=19, shape=(16, 16, 16), flags=lbm.LBM_FULL_ORDER) == 0
    assert "full_order" in lbm.lbm_last_error().lower()
    assert required(lattice=27, shape=(16, 16, 16), flags=lbm.LBM_FULL_ORDER) > 0
    assert required(lattice=9, shape=(16, 16, 1), flags=lbm.LBM_FULL_ORDER) > 0


def test_nested_box_validation():
    base = dict(lattice=9, shape=(48, 40, 1), refine_lo=(10, 8, 0), refine_hi=(36, 30, 0))
    assert lbm.lbm_required_bytes(lbm.make_config(nest=[((4, 4, 0), (20, 20, 0))], **base)) > 0
    # level 1 has 53 x 45 nodes: a box must lie in [4, n - 5]
    bad = lbm.make_config(nest=[((4, 4, 0), (49, 20, 0))], **base)
    assert lbm.lbm_required_bytes(bad) == 0
    assert "box 1" in lbm.lbm_last_error()
    cfg = lbm.make_config(lattice=9, shape=(48, 40, 1), nest=[((4, 4, 0), (20, 20, 0))])
    assert lbm.lbm_required_bytes(cfg) == 0


def test_comparator_collisions_validation():
    assert required(lattice=9, shape=(16, 16, 1), flags=lbm.LBM_MRT) > 0
    assert required(lattice=19, shape=(16, 16, 16), flags=lbm.LBM_MRT) == 0
    assert required(lattice=19, shape=(16, 16, 16), flags=lbm.LBM_BGK) > 0
    assert required(lattice=27, shape=(16, 16, 16), flags=lbm.LBM_BGK | lbm.LBM_FULL_ORDER) == 0
    assert required(lattice=9, shape=(16, 16, 1), flags=lbm.LBM_BGK | lbm.LBM_MRT) == 0
    assert required(lattice=9, shape=(32, 32, 1), flags=lbm.LBM_BGK, refine_lo=(8, 8, 0),
                    refine_hi=(20, 20, 0)) == 0
    assert required(lattice=9, shape=(32, 32, 1), flags=lbm.LBM_MRT, chi_max=0.1,
                    sponge_width=(0, 4, 0, 0, 0, 0), face_bc=(2, 2, 0, 0, 0, 0)) == 0


def test_moment_storage_validation_and_size():
    """Moment storages: ten values per cell (six on D2Q9) instead of q, and
    only on fully periodic, unrefined grids without a layer or comparator."""
    m = required(lattice=19, shape=(64, 64, 64), storage="m32")
    f = required(lattice=19, shape=(64, 64, 64), storage="f32")
    cells = 64 ** 3
    assert 10 * 4 * 2 * cells <= m < 10 * 4 * 2 * cells * 1.01 + (1 << 20)
    assert m < f * 0.6
    assert required(lattice=9, shape=(128, 128, 1), storage="m64") >= 6 * 8 * 2 * 128 * 128
    assert required(lattice=9, shape=(128, 128, 1), storage="m64") < 7 * 8 * 2 * 128 * 128 + (1 << 20)
    assert required(lattice=27, shape=(16, 16, 16), storage="m32", flags=lbm.LBM_FULL_ORDER) > 0
    bad = [dict(face_bc=(2, 2, 0, 0, 0, 0)),
           dict(refine_lo=(4, 4, 4), refine_hi=(12, 12, 12)),
           dict(chi_max=0.1, sponge_width=(4, 0, 0, 0, 0, 0)),
           dict(flags=lbm.LBM_SPONGE_FIELD),
           dict(flags=lbm.LBM_BGK)]
    for kw in bad:
        assert required(lattice=19, shape=(16, 16, 16), storage="m32", **kw) == 0, kw
        assert "moment storage" in lbm.lbm_last_error()


def test_halo_face_validation_and_size():
    """LBM_HALO (slab cut): last axis only, no refinement, no face layer on
    the cut, not with the moment storages; four buffers of the crossing
    populations of one face plane are added to the context."""
    base = dict(lattice=19, shape=(16, 12, 10), storage="f32")
    plain = required(**base)
    ring = required(face_bc=(0, 0, 0, 0, 3, 3), **base)
    assert ring - plain >= 4 * 5 * 16 * 12 * 4
    assert ring - plain < 4 * (5 * 16 * 12 * 4 + 256) + 1024
    assert required(face_bc=(2, 2, 1, 1, 3, 2), **base) > 0
    assert required(lattice=9, shape=(30, 20, 1), face_bc=(2, 2, 3, 1, 0, 0)) > 0
    bad = [(dict(face_bc=(3, 3, 0, 0, 0, 0)), "last axis"),
           (dict(face_bc=(0, 0, 3, 3, 0, 0)), "last axis"),
           (dict(lattice=9, shape=(30, 20, 1), face_bc=(3, 3, 0, 0, 0, 0)), "last axis"),
           (dict(face_bc=(0, 0, 0, 0, 3, 0)), "periodic"),
           (dict(face_bc=(0, 0, 0, 0, 3, 3), chi_max=0.1, sponge_width=(0, 0, 0, 0, 2, 0)),
            "absorbing layer"),
           (dict(face_bc=(2, 2, 2, 2, 3, 3), refine_lo=(4, 4, 4), refine_hi=(10, 8, 6)),
            "unrefined"),
           (dict(face_bc=(0, 0, 0, 0, 3, 3), storage="m32"), "moment storage"),
           (dict(face_bc=(0, 0, 0, 0, 4, 4)), "unknown rule")]
    for kw, msg in bad:
        cfg = dict(base)
        cfg.update(kw)
        assert required(**cfg) == 0, kw
        assert msg in lbm.lbm_last_error(), (kw, lbm.lbm_last_error())


def test_slab_split():
    from paper_1710_02065_amd.slabs import split
    assert split(10, 3) == [4, 3, 3]
    assert split(256, 8) == [32] * 8
    assert split(5, 5) == [1] * 5
    for n, k in [(4, 5), (4, 0)]:
        with pytest.raises(ValueError):
            split(n, k)
