"""Workspace sizing: the footprint entry points (kry_footprint,
kry_footprint_transposed) cover the bytes plan creation asks for,
and a workspace one byte short or misaligned is refused before any device
work (the plan's set-up queries the device first, so this runs on a GPU)."""
import ctypes as ct
import re

import pytest

import workloads as W
from gpu_helpers import require_gpu

pytestmark = pytest.mark.gpu


def _fake_csr_system(n):
    from paper_1804_01583_amd import kry
    s = kry.KrySystem()
    s.n = n
    s.kind = kry.KRY_CSR
    s.symmetric = 1
    s.rowptr = s.colidx = s.vals = 0x1000   # never dereferenced: every call here is refused first
    s.nnz = n
    return s



@pytest.mark.parametrize("route", ["forward", "transposed"])
def test_footprint_covers_what_plan_creation_needs(route):
    # every workspace here is misaligned and never dereferenced: creation
    # refuses a short one for its size (naming the bytes it needs) and one of
    # the footprint's size for its alignment, so no call reaches device work
    require_gpu()
    from paper_1804_01583_amd import kry
    keep = []
    s = _fake_csr_system(5000)
    bseg = kry._segs(W.segments_from_ranges([(10, 20)], 0.5), keep)
    s.b_segs = ct.pointer(bseg)
    gens = [W.Generator(W.segments_from_ranges([(0, 3)]), 0.0, 1.0),
            W.Generator(W.segments_from_ranges([(100, 140), (300, 310)]), 0.0, 1.0)]
    kg = [kry.KryGen(kry._segs(g.seg, keep), g.zc, g.radius) for g in gens]
    kc = [kry._segs(W.segments_from_ranges([(5, 9)]), keep), kry._segs(W.segments_from_ranges([(50, 90)]), keep)]
    k, steps, dt = 12, 30, 0.1
    nseg = sum(g.seg.nseg for g in gens) + 2 + 1
    if route == "forward":
        need = kry.kry_plan_workspace(s, len(gens) + 1, 2, k, steps, nseg)
        create = lambda ws, nb: kry.kry_plan_create(s, kg, None, kc, k, dt, steps, kry.KRY_FP64, kry.KRY_AUTO, 0,
                                                    ws, nb, None)
    else:
        need = kry.kry_footprint_transposed(s, len(gens), False, 2, k, steps, nseg)
        create = lambda ws, nb: kry.kry_plan_create_transposed(s, kg, None, kc, k, dt, steps, kry.KRY_FP64,
                                                               kry.KRY_AUTO, None, ws, nb)
    bad_ptr = 0x100008
    # a zero-byte workspace: refused for its size, naming the bytes needed
    with pytest.raises(kry.KryError) as ei:
        create(bad_ptr, 0)
    assert ei.value.status == kry.KRY_ENOMEM
    m = re.search(r"need (\d+) bytes", kry.lib.kry_last_error().decode())
    asked = int(m.group(1))
    # the footprint covers it (it may count a segment set's block table more)
    assert asked <= need <= asked + (64 << 10)
    with pytest.raises(kry.KryError) as ei:
        create(bad_ptr, asked - 1)
    assert ei.value.status == kry.KRY_ENOMEM
    with pytest.raises(kry.KryError) as ei:
        create(bad_ptr, need)
    assert ei.value.status == kry.KRY_EINVAL
    assert b"aligned" in kry.lib.kry_last_error()
