"""CPU checks of the C-ABI boundary: the built library exports every entry
point include/fastrsd.h declares, and host-only calls validate their
arguments (no GPU needed)."""

import ctypes
import math
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fastrsd.h")
LIB = os.path.join(ROOT, "paper_1506_02729_amd", "libfastrsd.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(frsd_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_function():
    assert os.path.exists(LIB), "library not built"
    names = declared_functions()
    assert len(names) >= 11
    lib = ctypes.CDLL(LIB)
    for n in names:
        assert hasattr(lib, n), n


def test_binding_covers_the_abi():
    from paper_1506_02729_amd import fastrsd as F
    assert set(declared_functions()) == set(F.EXPORTED)


def test_plan_validation_on_host():
    from paper_1506_02729_amd import fastrsd as F
    kf = 2 * math.pi / 500.0
    good = F.Config(n_grid=64, box=500.0, observer=(-300, -300, -300), order=2,
                    pk_dk=2 * kf, pk_nbins=16, max_objects=1000)
    h = F.frsd_plan_create(good.to_c())
    assert F.frsd_plan_workspace_bytes(h) > 64**3 * 8
    F.frsd_plan_destroy(h)
    bad = [
        dict(n_grid=100), dict(n_grid=16), dict(order=5), dict(ell_max=3), dict(precision=16),
        dict(pk_nbins=17),                     # beyond Nyquist
        dict(pk_dk=0.0), dict(box=-1.0),
        dict(bk_kmin=1.5 * kf, bk_dk=3 * kf, bk_nbins=11),   # bk beyond Nyquist
        dict(bk_kmin=1.5 * kf, bk_dk=3 * kf, bk_nbins=4, bk_grid=32),  # M too small
        dict(stream_slots=2),                  # slots without stream_moments
        dict(stream_moments=True, stream_slots=-1),
        dict(stream_moments=True, random_cache=True),
    ]
    for change in bad:
        cfg = F.Config(**{**good.__dict__, **change})
        with pytest.raises(F.FrsdError) as ei:
            F.frsd_plan_create(cfg.to_c())
        assert ei.value.code == F.FRSD_EINVAL, change
    # streamed plans: each resident slot adds its complex mesh and two assignment planes
    # (4 x 4 bytes x N^3 for FP32); slots beyond the 15 of the moments are clamped
    base = {**good.__dict__, "stream_moments": True, "ell_max": 4, "interlace": True}
    sizes = {k: F.workspace_bytes(F.Config(**{**base, "stream_slots": k})) for k in (1, 2, 3, 14, 15, 40)}
    assert sizes[2] == F.workspace_bytes(F.Config(**base))
    assert sizes[2] - sizes[1] == pytest.approx(16 * 64**3, abs=1024)
    assert sizes[3] - sizes[2] == pytest.approx(16 * 64**3, abs=1024)
    assert sizes[40] == sizes[15] > sizes[14]


def test_triangle_list_matches_oracle_rule():
    from oracle import estimator as est
    from paper_1506_02729_amd import fastrsd as F
    kf = 2 * math.pi / 3500.0
    cfg = F.Config(n_grid=256, box=3500.0, observer=(0, 0, 0), pk_dk=0.005, pk_nbins=40,
                   bk_kmin=1.5 * kf, bk_dk=3 * kf, bk_nbins=37, max_objects=10)
    h = F.frsd_plan_create(cfg.to_c())
    tri = F.frsd_bk_triangles(h)
    F.frsd_plan_destroy(h)
    prm = est.Params(n_grid=256, box=3500.0, observer=(0, 0, 0), bk_kmin=1.5 * kf, bk_dk=3 * kf, bk_nbins=37)
    ref = est.triangle_list(prm)
    assert tri.shape == ref.shape == (5416, 3)
    assert (tri == ref).all()


def test_triangle_grid_choice():
    """Default M is the smallest 2^a 3^b 5^c 7^d above 3 n_c (n_c = 112 for a
    top edge of 112.5 k_f); an explicit 7-smooth M is kept, other M rejected."""
    from paper_1506_02729_amd import fastrsd as F
    kf = 2 * math.pi / 3500.0
    base = dict(n_grid=256, box=3500.0, observer=(0, 0, 0), pk_dk=0.005, pk_nbins=40,
                bk_kmin=1.5 * kf, bk_dk=3 * kf, bk_nbins=37, max_objects=10)

    def smooth(m):
        for p in (2, 3, 5, 7):
            while m % p == 0:
                m //= p
        return m == 1

    expect = next(m for m in range(3 * 112 + 1, 2000) if smooth(m))
    assert expect == 343
    for bk_grid, want in ((0, expect), (350, 350), (360, 360), (384, 384)):
        h = F.frsd_plan_create(F.Config(**base, bk_grid=bk_grid).to_c())
        assert F.frsd_bk_grid(h) == want
        F.frsd_plan_destroy(h)
    for bad in (351, 336):   # a factor 13; below 3 n_c + 1
        with pytest.raises(F.FrsdError) as ei:
            F.frsd_plan_create(F.Config(**base, bk_grid=bad).to_c())
        assert ei.value.code == F.FRSD_EINVAL
    h = F.frsd_plan_create(F.Config(**{**base, "bk_nbins": 0}).to_c())
    assert F.frsd_bk_grid(h) == 0
    F.frsd_plan_destroy(h)


def test_workspace_shares_the_mesh_and_planar_regions():
    """The shell intermediates and fields (live only inside one bispectrum
    call) take the complex meshes and the planar assignment arrays (dead
    after the binning of frsd_pk_multipoles): at H512 the FP32 workspace with
    bispectrum bins is the P_ell-only one plus tables, the low-k cube and the
    contraction partials, and order 4 (PCS) plans build too."""
    from paper_1506_02729_amd import fastrsd as F
    kf = 2 * math.pi / 3500.0
    base = dict(n_grid=512, box=3500.0, observer=(-400.0, 1750.0, 1750.0), precision=32, pk_dk=0.005,
                pk_nbins=60, bk_kmin=1.5 * kf, bk_dk=3 * kf, bk_nbins=37, max_objects=41_000_000)
    h = F.frsd_plan_create(F.Config(**base).to_c())
    with_bk = F.frsd_plan_workspace_bytes(h)
    F.frsd_plan_destroy(h)
    h = F.frsd_plan_create(F.Config(**{**base, "bk_nbins": 0}).to_c())
    without_bk = F.frsd_plan_workspace_bytes(h)
    F.frsd_plan_destroy(h)
    meshes = 2 * 2 * 4 * 512**3 * 16         # 16 complex slots and their real/imaginary planes
    shells = 4 * 111 * 343**3                # 111 FP32 shell fields on M = 343
    assert shells < meshes
    assert with_bk - without_bk < 3e9        # tables, low-k cube and contraction partials only
    assert with_bk < 40e9
    h = F.frsd_plan_create(F.Config(**{**base, "order": 4}).to_c())
    F.frsd_plan_destroy(h)


def test_tuning_ranges_and_cache(tmp_path):
    """frsd_plan_set_tuning accepts the documented ranges only; the autotuner's
    JSON cache is keyed by plan shape and applied to plans of that shape."""
    import json
    from paper_1506_02729_amd import autotune
    from paper_1506_02729_amd import fastrsd as F
    kf = 2 * math.pi / 500.0
    cfg = F.Config(n_grid=64, box=500.0, observer=(-300, -300, -300), order=2, pk_dk=2 * kf, pk_nbins=16,
                   bk_kmin=1.5 * kf, bk_dk=3 * kf, bk_nbins=5, max_objects=1000)
    h = F.frsd_plan_create(cfg.to_c())
    assert F.frsd_plan_get_tuning(h) == {"tri_wg": 1024, "row_grid": 4096, "bin_blocks": 2048, "pair_batch": 8,
                                         "sweep_x": 0}
    good = {"tri_wg": 512, "row_grid": 2048, "bin_blocks": 4096, "pair_batch": 1, "sweep_x": 32}
    F.frsd_plan_set_tuning(h, good)
    assert F.frsd_plan_get_tuning(h) == good
    for bad in ({"tri_wg": 4096}, {"row_grid": 100}, {"bin_blocks": 8192}, {"pair_batch": 0}, {"pair_batch": 17},
                {"sweep_x": 8}, {"sweep_x": 48}, {"sweep_x": 128}):
        with pytest.raises(F.FrsdError) as ei:
            F.frsd_plan_set_tuning(h, dict(good, **bad))
        assert ei.value.code == F.FRSD_EINVAL
    assert F.frsd_plan_get_tuning(h) == good

    class FakePlan:
        pass
    fake = FakePlan()
    fake.cfg, fake.bk_grid, fake.handle = cfg, F.frsd_bk_grid(h), h
    path = tmp_path / "tuning.json"
    assert autotune.apply(fake, str(path)) is None
    want = {"tri_wg": 768, "row_grid": 8192, "bin_blocks": 1024, "pair_batch": 4, "sweep_x": 16}
    path.write_text(json.dumps({autotune.shape_key(cfg, fake.bk_grid): {"tuning": want}}))
    assert autotune.apply(fake, str(path)) == want
    assert F.frsd_plan_get_tuning(h) == want
    F.frsd_plan_destroy(h)


def test_ctypes_structs_match_the_c_header(tmp_path):
    """Every struct of the header has the size and field offsets the
    binding's ctypes mirror assumes (compiled with the host C compiler)."""
    import shutil
    import subprocess
    from paper_1506_02729_amd import fastrsd as F
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no host C compiler")
    structs = {"frsd_params": F.frsd_params, "frsd_tuning": F.frsd_tuning, "frsd_catalog": F.frsd_catalog,
               "frsd_pk_out": F.frsd_pk_out, "frsd_bk_out": F.frsd_bk_out}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "fastrsd.h"', "int main(void) {"]
    for name, cls in structs.items():
        lines.append(f'  printf("{name} sizeof %zu\\n", sizeof({name}));')
        for field, _ in cls._fields_:
            lines.append(f'  printf("{name} {field} %zu\\n", offsetof({name}, {field}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "abi.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "abi"
    subprocess.run([cc, "-std=c99", "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    got = {}
    for line in subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.splitlines():
        name, field, val = line.split()
        got[(name, field)] = int(val)
    for name, cls in structs.items():
        assert got[(name, "sizeof")] == ctypes.sizeof(cls), name
        for field, _ in cls._fields_:
            assert got[(name, field)] == getattr(cls, field).offset, (name, field)


def test_batch_validation_on_host():
    """frsd_pk_batch checks every request before any device work: batch size,
    plans of one shape, distinct plans and workspaces, initialised workspaces."""
    from paper_1506_02729_amd import fastrsd as F
    kf = 2 * math.pi / 500.0
    base = dict(n_grid=64, box=500.0, observer=(-300, -300, -300), order=2, pk_dk=2 * kf, pk_nbins=16,
                max_objects=1000)
    hs = [F.frsd_plan_create(F.Config(**base).to_c()) for _ in range(3)]
    other = F.frsd_plan_create(F.Config(**{**base, "order": 3}).to_c())
    ws = [256 * (k + 1) for k in range(4)]  # aligned placeholders: never dereferenced
    gal = F.frsd_catalog()
    out = F.frsd_pk_out()

    def call(plans, wss):
        n = len(plans)
        F.frsd_pk_batch(plans, wss, [gal] * n, None, [1.0] * n, [out] * n, None)

    def call_empty():
        F._check(F._lib.frsd_pk_batch((F._P * 1)(hs[0]), (F._P * 1)(ws[0]), 0, (F.frsd_catalog * 1)(gal), None,
                                      (ctypes.c_double * 1)(1.0), (F.frsd_pk_out * 1)(out), None))

    try:
        cases = [
            (call_empty, F.FRSD_EINVAL),                                       # empty batch
            (lambda: call(hs[:2] + [other], ws[:3]), F.FRSD_EINVAL),           # plans of two shapes
            (lambda: call([hs[0], hs[1]], [ws[0], ws[0]]), F.FRSD_EINVAL),    # one workspace twice
            (lambda: call([hs[0], hs[0]], ws[:2]), F.FRSD_EINVAL),            # one plan twice
            (lambda: call(hs, [ws[0], ws[1] + 8, ws[2]]), F.FRSD_EINVAL),     # misaligned workspace
            (lambda: call(hs, ws[:3]), F.FRSD_ESTATE),                         # not initialised
        ]
        for fn, code in cases:
            with pytest.raises(F.FrsdError) as ei:
                fn()
            assert ei.value.code == code, F.frsd_last_error()
        # graph capture of a batch: randoms required, an explicit stream required, the batch checks as above
        with pytest.raises(F.FrsdError) as ei:
            F._check(F._lib.frsd_graph_create_batch((F._P * 2)(*hs[:2]), (F._P * 2)(*ws[:2]), 2,
                                                    (F.frsd_catalog * 2)(gal, gal), None,
                                                    (ctypes.c_double * 2)(1.0, 1.0), (F.frsd_pk_out * 2)(out, out),
                                                    None, ctypes.byref(F._P())))
        assert ei.value.code == F.FRSD_EINVAL
        with pytest.raises(F.FrsdError) as ei:
            F.frsd_graph_create_batch(hs[:2], ws[:2], [gal] * 2, [gal] * 2, [1.0] * 2, [out] * 2, None)
        assert ei.value.code == F.FRSD_EINVAL  # null stream
        with pytest.raises(F.FrsdError) as ei:
            F.frsd_graph_launch_batch(None, [1], [1], [1.0], None)
        assert ei.value.code == F.FRSD_EINVAL
        big = [gal] * (F.FRSD_MAX_BATCH + 1)
        with pytest.raises(F.FrsdError) as ei:
            F.frsd_pk_batch([hs[0]] * len(big), [ws[0]] * len(big), big, None, [1.0] * len(big),
                            [out] * len(big), None)
        assert ei.value.code == F.FRSD_EINVAL
    finally:
        for h in hs + [other]:
            F.frsd_plan_destroy(h)


def test_batch_server_arguments():
    """BatchServer refuses group sizes beyond a batch and a shared random
    catalogue on a configuration without the random cache (before any
    device work)."""
    from paper_1506_02729_amd import fastrsd as F
    from paper_1506_02729_amd.serve import BatchServer
    kf = 2 * math.pi / 500.0
    cfg = F.Config(n_grid=64, box=500.0, observer=(-300, -300, -300), order=2, pk_dk=2 * kf, pk_nbins=16,
                   max_objects=1000)
    for size in (0, F.FRSD_MAX_BATCH + 1):
        with pytest.raises(ValueError):
            BatchServer(cfg, group_size=size)
    with pytest.raises(ValueError):
        BatchServer(cfg, randoms={"pos": None, "w": None, "nbar": None})
