"""The C ABI: liblbmd.so loads on a host without a GPU, exports every entry
point include/lbmd.h declares, and validates descriptions on the host
(lb_buffer_sizes calls no HIP function)."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = []
    for h in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if not h.endswith(".h"):
            continue
        txt = open(os.path.join(ROOT, "include", h)).read()
        txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
        names += re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s+\**\s*([a-z_][a-z0-9_]*)\s*\(",
                            txt, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = _declared()
    for n in ("lb_buffer_sizes", "lb_init", "lb_step", "md_couple_step", "lb_observables", "lb_destroy",
              "lb_get_state", "lb_set_state", "lb_check", "lb_last_error", "md_relax"):
        assert n in names, n


def test_library_exports_every_declared_symbol():
    from paper_0711_2665_amd import lbmd
    L = lbmd.lib()
    missing = [n for n in _declared() if not hasattr(L, n)]
    assert not missing, missing


def test_desc_layout_matches_header(tmp_path):
    # the ctypes mirrors have the size and the field offsets the C compiler
    # gives the structs of include/lbmd.h
    from paper_0711_2665_amd import lbmd
    structs = {"lb_desc": lbmd.LbDesc, "lb_sizes": lbmd.LbSizes, "lb_buffers": lbmd.LbBuffers}
    lines = ['#include <stdio.h>', '#include "lbmd.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'  printf("{cname} sizeof %zu\\n", sizeof({cname}));')
        for f in py._fields_:
            lines.append(f'  printf("{cname} {f[0]} %zu\\n", offsetof({cname}, {f[0]}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    import subprocess
    subprocess.check_call(["gcc", "-std=c99", "-I" + os.path.join(ROOT, "include"), "-o", str(exe), str(src)])
    got = {}
    for ln in subprocess.check_output([str(exe)], text=True).splitlines():
        cname, field, val = ln.split()
        got[(cname, field)] = int(val)
    for cname, py in structs.items():
        assert got[(cname, "sizeof")] == C.sizeof(py), cname
        for f in py._fields_:
            assert got[(cname, f[0])] == getattr(py, f[0]).offset, (cname, f[0])
    assert {f[0] for f in lbmd.LbDesc._fields_} >= {"fluid_kT", "seed", "replica"}


@pytest.mark.parametrize("bad,msg", [
    (dict(tau=0.5), "tau"),
    (dict(shape=(0, 4, 4)), "extents"),
    (dict(wall_axis=2, wall_pos=1), "wall plane"),
    (dict(wall_axis=2, wall_pos=8, pore_h=40), "pore"),
    (dict(n_sub=0), "n_sub"),
    (dict(nb=-1), "negative"),
    (dict(nb=3, mass=0.0), "mass"),
    (dict(nb=3, mass=2.0, gamma=0.1), "mass 1"),
    (dict(nb=3, rc=3.5), "rc"),
    (dict(nb=3, wall_axis=2, wall_pos=2, shape=(16, 5, 8)), "extents >= 6"),
    (dict(shape=(1024, 1024, 128)), "too large"),
    (dict(fluid_kT=-1e-4), "fluid_kT"),
    (dict(mts_outer=3), "mts_outer"),
    (dict(mts_outer=1), "mts_outer"),
    (dict(mts_outer=-1), "mts_outer"),
    (dict(coupling=2), "coupling"),
    (dict(constraints=2), "constraints"),
    (dict(constraints=1, nb=2000, shape=(64, 64, 64)), "rigid bonds"),
    (dict(constraints=1, mts_outer=5), "rigid bonds"),
])
def test_host_validation(bad, msg):
    from paper_0711_2665_amd import lbmd
    from paper_0711_2665_amd.workloads import BASE
    cfg = dict(BASE)
    cfg.update(shape=(16, 16, 16), wall_axis=-1, wall_pos=0, pore_h=0, nb=0)
    cfg.update(bad)
    with pytest.raises(lbmd.LbError) as e:
        lbmd.buffer_sizes(cfg)
    assert e.value.code == lbmd.LB_ERR_ARG
    assert msg in str(e.value)


def test_unit_mass_needed_only_with_friction():
    # the exponential kick's friction term is exact only at unit mass; an
    # uncoupled chain (gamma = 0) may carry any positive mass
    from paper_0711_2665_amd import lbmd
    from paper_0711_2665_amd.workloads import BASE
    cfg = dict(BASE)
    cfg.update(shape=(16, 16, 16), wall_axis=-1, wall_pos=0, pore_h=0, nb=3, mass=2.0, gamma=0.0)
    lbmd.buffer_sizes(cfg)


def test_buffer_sizes_are_aligned_and_exact():
    from paper_0711_2665_amd import lbmd
    from paper_0711_2665_amd.workloads import C3
    s = lbmd.buffer_sizes(C3, lbmd.LB_FP32_DEV)
    N = 512 * 256 * 256
    assert s["pops_bytes"] == 19 * N * 4
    assert s["flags_bytes"] == N
    assert all(v % 256 == 0 for k, v in s.items() if k.endswith("_bytes"))
    assert s["nodes"] == N and s["bead_slots"] == 8000
    assert s["snapshot_bytes"] >= s["pops_bytes"] + s["force_bytes"] + s["beads_bytes"] + s["work_bytes"]
    s64 = lbmd.buffer_sizes(C3, lbmd.LB_FP64)
    assert s64["pops_bytes"] == 19 * N * 8


def test_ensemble_sizes_pack_replicas():
    """Host-only packing of an uneven ensemble: node offsets rounded to 64
    nodes, bead slots to 16 per chain; mixed n_sub is refused."""
    from paper_0711_2665_amd import lbmd
    from paper_0711_2665_amd.workloads import C0, scaled
    cfgs = [scaled(C0, shape=(16, 12, 20), wall_pos=10, nb=12), scaled(C0, shape=(12, 12, 13), wall_axis=-1,
                                                                          wall_pos=0, pore_h=0, nb=0),
            scaled(C0, shape=(24, 24, 24), wall_pos=12, nb=33)]
    s = lbmd.ensemble_sizes(cfgs, lbmd.LB_FP32_DEV)
    nodes = 3840 + 1920 + 13824
    assert s["nodes"] == nodes and s["bead_slots"] == 16 + 0 + 48
    assert s["pops_bytes"] == (19 * nodes * 4 + 255) // 256 * 256
    with pytest.raises(lbmd.LbError) as e:
        lbmd.ensemble_sizes([cfgs[0], scaled(cfgs[2], n_sub=50)])
    assert "n_sub" in str(e.value)
    with pytest.raises(lbmd.LbError) as e:
        lbmd.ensemble_sizes([cfgs[0], dict(cfgs[2], tau=0.4)])
    assert "replica 1" in str(e.value)



def test_binding_direction_order_is_the_oracles(orc):
    """The binding's D3Q19 table (the header's documented storage order) is
    the oracle's; the GPU parity tests compare populations index by index
    with the oracle, so it is also the library's."""
    import numpy as np
    from paper_0711_2665_amd import lbmd
    c, w, opp = orc.tables()
    assert np.array_equal(np.asarray(lbmd.VELOCITIES, dtype=np.float64), np.asarray(c, dtype=np.float64))
    assert np.array_equal(np.asarray(lbmd.WEIGHTS), np.asarray(w))
    # the header's text lists the same order
    hdr = open(os.path.join(os.path.dirname(__file__), "..", "include", "lbmd.h")).read()
    for i, ci in enumerate(lbmd.VELOCITIES):
        if sum(abs(x) for x in ci) == 2:
            assert "(" + ",".join(str(x) for x in ci) + ")" in hdr.replace(" ", ""), (i, ci)
