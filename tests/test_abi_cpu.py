"""Host-side checks of the C ABI (no GPU needed): the library loads, exports every
symbol the header declares, validates descriptors exactly as documented and
plans the expected launch schedules."""
import ctypes
import os
import re

import pytest

from paper_1309_0392_amd import sgh
from paper_1309_0392_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sgh.h")


def header_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sgh_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = sgh.lib()
    names = header_functions()
    assert len(names) >= 18
    for name in names:
        assert hasattr(lib, name), name


def test_header_constants_match_binding():
    text = open(HEADER).read()
    consts = dict(re.findall(r"#define (SGH_[A-Z0-9_]+) \(?(-?\w+)\)?", text))
    assert int(consts["SGH_MAX_DIM"]) == sgh.MAX_DIM
    assert int(consts["SGH_MAX_LEVEL"]) == sgh.MAX_LEVEL
    assert int(consts["SGH_F32"]) == sgh.F32 and int(consts["SGH_F64"]) == sgh.F64
    assert int(consts["SGH_ERR_OVERLAP"]) == sgh.ERR_OVERLAP
    assert int(consts["SGH_PLAN_GRAPH"].rstrip("u")) == sgh.PLAN_GRAPH
    assert int(consts["SGH_PLAN_RELATIVE"].rstrip("u")) == sgh.PLAN_RELATIVE
    assert int(consts["SGH_STATIC_TASKS"]) == sgh.STATIC_TASKS
    # struct layout: dim, level[16], dtype, data pointer
    assert ctypes.sizeof(sgh.SghGrid) == 80 and sgh.SghGrid.data.offset == 72


def fake(levels, dtype=sgh.F64, ptr=0x10000):
    return sgh.make_grid(levels, dtype, ptr)


def test_validation_codes():
    v = sgh.validate
    assert v([]) == sgh.OK
    assert v([fake((5, 5))]) == sgh.OK
    assert v([fake((5, 5), ptr=0)]) == sgh.ERR_ARG                     # null data
    g = fake((5, 5)); g.dim = 0
    assert v([g]) == sgh.ERR_ARG                                        # dim 0
    g = fake((5, 5)); g.dim = 17
    assert v([g]) == sgh.ERR_ARG                                        # dim > max
    assert v([fake((0, 3))]) == sgh.ERR_ARG                             # level 0
    assert v([fake((31,))]) == sgh.ERR_ARG                              # level > 30
    assert v([fake((20, 20, 20))]) == sgh.ERR_ARG                       # size overflow
    assert v([fake((5, 5), dtype=7)]) == sgh.ERR_DTYPE
    assert v([fake((5, 5), ptr=0x10004)]) == sgh.ERR_ALIGN              # f64 at 4-byte offset
    assert v([fake((5, 5), dtype=sgh.F32, ptr=0x10004)]) == sgh.OK
    n_bytes = 31 * 31 * 8
    assert v([fake((5, 5), ptr=0x10000), fake((5, 5), ptr=0x10000 + n_bytes)]) == sgh.OK
    assert v([fake((5, 5), ptr=0x10000), fake((5, 5), ptr=0x10000 + n_bytes - 8)]) == sgh.ERR_OVERLAP
    assert sgh.lib().sgh_validate(None, -1) == sgh.ERR_ARG
    assert sgh.lib().sgh_validate(None, 1) == sgh.ERR_ARG
    assert "level" in sgh.last_error_message() or "grid" in sgh.last_error_message()


def test_transform_rejects_before_launch():
    """Invalid descriptors come back as codes without touching a device."""
    bad = sgh.grid_array([fake((5, 5)), fake((0, 5))])
    assert sgh.lib().sgh_hierarchize(bad, 2, None) == sgh.ERR_ARG
    assert sgh.lib().sgh_transform(3, bad, 0, None) == sgh.ERR_ARG      # unknown op
    plan = ctypes.c_void_p()
    assert sgh.lib().sgh_plan_create(ctypes.byref(plan), 0, bad, 2, 0) == sgh.ERR_ARG
    assert plan.value is None
    assert sgh.lib().sgh_plan_create(None, 0, bad, 0, 0) == sgh.ERR_ARG


def test_error_strings_and_version():
    for code in (0, -1, -2, -3, -4, -5, -6, -7, -99):
        assert isinstance(sgh.error_string(code), str) and sgh.error_string(code)
    assert re.match(r"\d+\.\d+\.\d+", sgh.version())


def test_num_points():
    assert sgh.num_points(W.SMALL_2D) == 961
    assert sgh.num_points(W.ANISO_3D) == 133302015
    assert sgh.num_points(W.ANISO_5D) == 118240479
    assert sgh.num_points((0,)) == -1


def test_schedules():
    # in place: axis 0 in an LDS tile fused with axis 1 walked in registers
    # (each workgroup streams one contiguous plane); axis 2 strided
    s = sgh.schedule(sgh.OP_HIERARCHIZE, W.ANISO_3D)
    kinds = [(l["kind"], tuple(l["axes"])) for l in s["launches"]]
    assert kinds == [("tw", (0, 1)), ("pole", (2,))]
    assert [l.get("L") for l in s["launches"]] == [9, 8]
    assert [(l["split"], l["TB"], l["B"]) for l in s["launches"]] == [(3, 3, 3), (3, 2, 3)]
    assert s["launches"][1]["prefetch"] == 1 and s["launches"][0]["outer_level"] == 0
    assert s["hbm_round_trips"] == 2
    # out of place the hierarchization also folds axis 2 (its one-shot stencil
    # applied as each plane's rows are read): one launch
    so = sgh.schedule(sgh.OP_HIERARCHIZE, W.ANISO_3D, out_of_place=True)
    assert [(l["kind"], tuple(l["axes"])) for l in so["launches"]] == [("tw", (0, 1, 2))]
    assert (so["launches"][0]["L"], so["launches"][0]["outer_level"]) == (9, 8)
    assert so["hbm_round_trips"] == 1
    try:
        sgh.set_outer_stencil(0)
        so = sgh.schedule(sgh.OP_HIERARCHIZE, W.ANISO_3D, out_of_place=True)
        assert [(l["kind"], tuple(l["axes"])) for l in so["launches"]] == [("tw", (0, 1)), ("pole", (2,))]
    finally:
        sgh.set_outer_stencil(1)
    with pytest.raises(sgh.SghError):
        sgh.set_outer_stencil(2)
    # only the hierarchization has the one-shot stencil, only out of place; a
    # two-level walk folds nothing
    for lv in ((10, 9, 8), (10, 7, 3, 2), (9, 8, 5)):
        for op in (sgh.OP_HIERARCHIZE, sgh.OP_DEHIERARCHIZE, sgh.OP_ADJOINT):
            assert all(l.get("outer_level", 0) == 0 for l in sgh.schedule(op, lv)["launches"])
            if op != sgh.OP_HIERARCHIZE:
                assert all(l.get("outer_level", 0) == 0
                           for l in sgh.schedule(op, lv, out_of_place=True)["launches"])
    assert [tuple(l["axes"]) for l in sgh.schedule(sgh.OP_HIERARCHIZE, (10, 7, 3, 2), out_of_place=True)[
        "launches"]] == [(0, 1, 2), (3,)]
    assert sgh.schedule(sgh.OP_HIERARCHIZE, (10, 4, 8), out_of_place=True)["launches"][0]["outer_level"] == 0
    d = sgh.schedule(sgh.OP_DEHIERARCHIZE, W.ANISO_3D)
    assert [tuple(l["axes"]) for l in d["launches"]] == [(2,), (0, 1)]
    s5 = sgh.schedule(sgh.OP_HIERARCHIZE, W.ANISO_5D)
    assert [(l["kind"], tuple(l["axes"])) for l in s5["launches"]] == [
        ("tw", (0, 1, 2)), ("pole", (3,)), ("pole", (4,))]
    assert s5["launches"][0]["ept"] == 4 and s5["launches"][0]["tile"] == 63 * 63
    small = sgh.schedule(sgh.OP_HIERARCHIZE, W.SMALL_2D)
    assert [(l["kind"], tuple(l["axes"])) for l in small["launches"]] == [("tile", (0, 1))]
    # level-1 axes are the identity and are dropped
    assert sgh.schedule(sgh.OP_HIERARCHIZE, (1, 1))["launches"] == []
    # long poles use the dyadic split: a contiguous l=14 pole is 4 blocks of
    # 2^12 positions (FP64: 32 KiB tiles), then the level-2 lattice of the
    # block boundaries
    lv = sgh.schedule(sgh.OP_HIERARCHIZE, (14,))["launches"]
    assert [(l["kind"], l["E"], l["Bs"], l["W"]) for l in lv] == [("split", 0, 12, 1), ("split", 12, 2, 1)]
    lv = sgh.schedule(sgh.OP_ADJOINT, (14,))["launches"]
    assert [(l["E"], l["Bs"]) for l in lv] == [(12, 2), (0, 12)]
    # l=27 (1 GiB FP64): fine blocks of 2^12, then the level-15 coarse pole in
    # blocks of 2^7 lattice steps, then the level-8 lattice, then the root
    # (which only the transpose changes)
    for op, order in ((sgh.OP_HIERARCHIZE, [0, 12, 19]), (sgh.OP_DEHIERARCHIZE, [19, 12, 0]),
                      (sgh.OP_ADJOINT, [26, 19, 12, 0])):
        lv = sgh.schedule(op, (27,))["launches"]
        assert [l["E"] for l in lv] == order
    # FP32 tiles hold twice the positions
    lv = sgh.schedule(sgh.OP_HIERARCHIZE, (27,), sgh.F32)["launches"]
    assert [(l["E"], l["Bs"]) for l in lv] == [(0, 13), (13, 7), (20, 7)]
    try:
        sgh.set_split_spans(12, 8)
        lv = sgh.schedule(sgh.OP_HIERARCHIZE, (27,))["launches"]
        assert [(l["E"], l["Bs"]) for l in lv] == [(0, 12), (12, 8), (20, 7)]
        sgh.set_split_spans(16, 0)  # capped to what fits the tile
        assert sgh.schedule(sgh.OP_HIERARCHIZE, (27,))["launches"][0]["Bs"] == 13
    finally:
        sgh.set_split_spans(0, 0)
    with pytest.raises(sgh.SghError):
        sgh.set_split_spans(-1, 0)
    # a strided long axis: 32 adjacent poles per workgroup (stride 31), blocks of 2^7
    lv = sgh.schedule(sgh.OP_ADJOINT, (5, 12))["launches"]
    assert [(l["kind"], l.get("E"), l.get("Bs"), l.get("W")) for l in lv] == [
        ("split", 7, 5, 32), ("split", 0, 7, 32), ("tile", None, None, None)]
    # a walked axis that is not the last one (the last is too long for registers)
    lv = sgh.schedule(sgh.OP_HIERARCHIZE, (10, 4, 11))["launches"]
    assert [(l["kind"], tuple(l["axes"])) for l in lv] == [("tw", (0, 1)), ("split", (2,)), ("split", (2,))]
    assert sgh.schedule(sgh.OP_HIERARCHIZE, (10, 4, 11))["hbm_round_trips"] == 2
    lv = sgh.schedule(sgh.OP_HIERARCHIZE, (10, 11, 4))["launches"]
    assert [(l["kind"], tuple(l["axes"])) for l in lv][0] == ("tw", (0, 2))


def test_box_schedules():
    # the 10-dimensional anisotropic shape: the first axis refined, nine axes of 3 points
    ten = (12,) + (2,) * 9
    s = sgh.schedule(sgh.OP_HIERARCHIZE, ten)
    assert [(l["kind"], tuple(l["axes"])) for l in s["launches"]] == [
        ("tw", (0, 1)), ("box", (2, 3, 4, 5, 6)), ("box", (7, 8, 9))]
    assert [l.get("W") for l in s["launches"]] == [None, 32, 64] and s["hbm_round_trips"] == 3
    d = sgh.schedule(sgh.OP_DEHIERARCHIZE, ten)
    assert [tuple(l["axes"]) for l in d["launches"]] == [(7, 8, 9), (2, 3, 4, 5, 6), (0, 1)]
    # boxes stay within the limits; a single small axis keeps its pole launch
    try:
        sgh.set_box_limits(16384, 256)
        s = sgh.schedule(sgh.OP_HIERARCHIZE, ten)
        assert [len(l["axes"]) for l in s["launches"]] == [2, 3, 3, 2]
        assert all(l["box"] * 8 <= 16384 and l["W"] * 8 >= 256 for l in s["launches"] if l["kind"] == "box")
    finally:
        sgh.set_box_limits(0, 0)
    assert [l["kind"] for l in sgh.schedule(sgh.OP_DEHIERARCHIZE, (10, 9, 8))["launches"]] == ["pole", "tw"]
    # FP32 rows of 16 columns are too short to pair the two level-5 axes of (6,6,5,5,5)
    s = sgh.schedule(sgh.OP_HIERARCHIZE, W.ANISO_5D, sgh.F32)
    assert [l["kind"] for l in s["launches"]] == ["tw", "pole", "pole"]
    # fusion level 0: one launch per strided axis
    try:
        sgh.set_fusion(0)
        assert "box" not in [l["kind"] for l in sgh.schedule(sgh.OP_HIERARCHIZE, ten)["launches"]]
    finally:
        sgh.set_fusion(1)
    with pytest.raises(sgh.SghError):
        sgh.set_box_limits(-1, 0)


def test_box_limits_whole_range_launchable():
    # every box the knob's accepted range can form has a kernel instantiation:
    # 256 or 512 threads of 4..32 elements covering the box
    shapes = [(13, 3, 3, 3, 3), (12,) + (2,) * 9, (4, 5, 5, 5), (2,) * 12, (6, 6, 5, 5, 5), (3, 2, 4, 3, 2, 5)]
    try:
        for max_bytes in list(range(0, 160 * 1024 + 1, 4096)) + [160 * 1024]:
            for row in (0, 16, 64, 128, 512):
                sgh.set_box_limits(max_bytes, row)
                for lv in shapes:
                    for dt in (sgh.F32, sgh.F64):
                        for op in (sgh.OP_HIERARCHIZE, sgh.OP_ADJOINT):
                            for l in sgh.schedule(op, lv, dt)["launches"]:
                                if l["kind"] != "box":
                                    continue
                                assert l["nt"] in (256, 512) and l["ept"] in (4, 8, 16, 32), (max_bytes, row, lv, l)
                                assert l["box"] <= l["nt"] * l["ept"], (max_bytes, row, lv, l)
    finally:
        sgh.set_box_limits(0, 0)


def test_fusion_switch():
    try:
        sgh.set_fusion(0)
        s = sgh.schedule(sgh.OP_HIERARCHIZE, W.ANISO_3D)
        assert [(l["kind"], tuple(l["axes"])) for l in s["launches"]] == [
            ("tile", (0,)), ("pole", (1,)), ("pole", (2,))]
        d = sgh.schedule(sgh.OP_ADJOINT, W.ANISO_3D)
        assert [tuple(l["axes"]) for l in d["launches"]] == [(2,), (1,), (0,)]
    finally:
        sgh.set_fusion(1)
    with pytest.raises(sgh.SghError):
        sgh.set_fusion(5)
    assert sgh.schedule(sgh.OP_HIERARCHIZE, W.ANISO_3D)["launches"][0]["kind"] == "tw"
    with pytest.raises(sgh.SghError):
        sgh.set_pole_block(9, 7)
    with pytest.raises(sgh.SghError):
        sgh.set_pole_split(9, 1, 4, 0)
    try:
        sgh.set_fusion(2)
        s = sgh.schedule(sgh.OP_HIERARCHIZE, W.ANISO_3D)
        assert (s["launches"][0]["kind"], s["launches"][0]["split"]) == ("tw", 2)
        sgh.set_pole_split(9, 3, 3, 1)
        s = sgh.schedule(sgh.OP_HIERARCHIZE, W.ANISO_3D)
        assert (s["launches"][1]["split"], s["launches"][1]["prefetch"]) == (3, 1)
    finally:
        sgh.set_fusion(1)
        sgh.set_pole_split(9, 0, 0, 0)


def test_batch_classes_knob():
    sgh.set_batch_classes(0, 1)
    sgh.set_batch_classes(10, 5)
    sgh.set_batch_classes()
    for bad in ((-1, 1), (4096, 0), (4096, 1, 2)):
        with pytest.raises(sgh.SghError):
            sgh.set_batch_classes(*bad)


def test_transform_out_validation():
    # rejected on the host before anything is launched (no device needed)
    import ctypes
    src = sgh.grid_array([fake((5, 5), ptr=0x100000)])
    bad = [(fake((5, 5), ptr=0x100000 + 8 * 100), sgh.ERR_OVERLAP),   # overlaps the source
           (fake((5, 4), ptr=0x200000), sgh.ERR_ARG),                   # other shape
           (fake((5, 5), dtype=sgh.F32, ptr=0x200000), sgh.ERR_ARG),    # other dtype
           (fake((5, 5), ptr=0x200004), sgh.ERR_ALIGN)]
    for g, code in bad:
        assert sgh.lib().sgh_transform_out(0, src, sgh.grid_array([g]), 1, None) == code
    two_src = sgh.grid_array([fake((3,), ptr=0x100000), fake((3,), ptr=0x101000)])
    # destination 0 on top of source 1
    two_dst = sgh.grid_array([fake((3,), ptr=0x101000), fake((3,), ptr=0x300000)])
    assert sgh.lib().sgh_transform_out(0, two_src, two_dst, 2, None) == sgh.ERR_OVERLAP
    assert sgh.lib().sgh_transform_out(7, src, src, 1, None) == sgh.ERR_ARG
    assert sgh.lib().sgh_transform_out(0, src, src, 0, None) == sgh.OK  # nothing to do


def test_static_batch_rejects_too_many_grids_before_launch():
    # more small grids than the fixed device task array holds: refused on the
    # host before any device call (no device needed)
    n = sgh.STATIC_TASKS + 1
    grids = sgh.grid_array([fake((2,), ptr=0x100000 + 64 * i) for i in range(n)])
    assert sgh.lib().sgh_transform_batch_static(0, grids, n, None) == sgh.ERR_UNSUPPORTED
    assert "at most %d" % sgh.STATIC_TASKS in sgh.last_error_message()
    assert sgh.lib().sgh_transform_batch_static(5, grids, 1, None) == sgh.ERR_ARG


def test_plain_descriptor_may_not_be_null():
    # (a relative plan's offsets may be 0; plain descriptors need a pointer)
    assert sgh.validate([sgh.make_grid((5, 5), sgh.F64, 0)]) == sgh.ERR_ARG


def test_medium_limits_knob():
    sgh.set_medium_limits(0, 1)  # 0 turns the medium launch off
    sgh.set_medium_limits(1 << 24, 100)
    sgh.set_medium_limits()
    for bad in ((-1, 16), ((1 << 24) + 1, 16), (1 << 18, 0)):
        with pytest.raises(sgh.SghError):
            sgh.set_medium_limits(*bad)
