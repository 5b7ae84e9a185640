"""The C-ABI library loads on the CPU and exports every entry point include/efpi.h declares,
and its host-side argument checks reject bad configurations without touching a GPU."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "efpi.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(efpi_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    import paper_1610_01071_amd.efpi as E
    names = declared_functions()
    assert len(names) >= 20
    for n in names:
        assert hasattr(E.LIB, n), n
        assert n in E.EXPORTED, n


def test_binding_struct_layout_matches_header():
    import ctypes
    import paper_1610_01071_amd.efpi as E
    # efpi_replica: 8 int32, 5 double, 1 int64, then the electron fields
    # 2 double, 2 int32, 1 int64 -> 80 + 32 = 112 bytes
    assert ctypes.sizeof(E.Replica) == 112
    assert E.Replica.length.offset == 32 and E.Replica.capacity.offset == 72
    assert E.Replica.qm_e.offset == 80 and E.Replica.ppc_e.offset == 96
    assert E.Replica.capacity_e.offset == 104
    # efpi_config: 2 uint32, pointer, 2 int32, double, 2 int32, uint32 (+ padding)
    assert E.Config.replicas.offset == 8 and E.Config.newton_tol.offset == 24


@pytest.mark.parametrize("field,value,msg", [
    ("n_cells", 100, "power of two"),
    ("n_cells", 32768, "power of two"),
    ("haar_levels", 12, "haar_levels"),
    ("dt", 0.0, "dt"),
    ("macro_dt", 0.5, "macro_dt"),
    ("ppc", 0, "ppc"),
    ("closure", 3, "closure"),
    ("capacity", -5, "capacity"),
])
def test_config_validation(field, value, msg):
    import paper_1610_01071_amd.efpi as E
    spec = E.ReplicaSpec(1024, 1024.0, ppc=10)
    cfg = E.ConfigSpec([spec]).to_c()
    setattr(cfg.replicas[0], field, value)
    with pytest.raises(E.EfpiError) as ei:
        E.efpi_workspace_size(cfg)
    assert ei.value.status == -1 and msg in str(ei.value)


@pytest.mark.parametrize("field,value,msg", [
    ("bc", 1, "periodic"),
    ("n_cells", 16384, "8192"),
    ("qm_e", 1.0, "qm_e"),
    ("vth_e", -1.0, "vth_e"),
    ("ppc_e", 0, "ppc_e"),
    ("pad_e", 3, "pad_e"),
    ("capacity_e", 0, "capacity_e"),
])
def test_kinetic_config_validation(field, value, msg):
    import paper_1610_01071_amd.efpi as E
    spec = E.ReplicaSpec(1024, 1024.0, ppc=10, closure=E.CLOSURE_KINETIC, ppc_e=10)
    cfg = E.ConfigSpec([spec]).to_c()
    E.efpi_workspace_size(cfg)
    setattr(cfg.replicas[0], field, value)
    with pytest.raises(E.EfpiError) as ei:
        E.efpi_workspace_size(cfg)
    assert ei.value.status == -1 and msg in str(ei.value)


def test_kinetic_replicas_not_mixed():
    import paper_1610_01071_amd.efpi as E
    specs = [E.ReplicaSpec(256, 256.0, ppc=10, closure=E.CLOSURE_KINETIC, ppc_e=10),
             E.ReplicaSpec(256, 256.0, ppc=10)]
    with pytest.raises(E.EfpiError) as ei:
        E.efpi_workspace_size(E.ConfigSpec(specs).to_c())
    assert "every replica" in str(ei.value)


def test_kinetic_workspace_holds_the_electron_store():
    import paper_1610_01071_amd.efpi as E
    a = E.efpi_workspace_size(E.ConfigSpec([E.ReplicaSpec(4096, 4096.0, ppc=100)]).to_c())
    b = E.efpi_workspace_size(E.ConfigSpec([E.ReplicaSpec(
        4096, 4096.0, ppc=100, closure=E.CLOSURE_KINETIC, ppc_e=300)]).to_c())
    # 14 bytes per electron slot plus the electron loading arrays (< 200 KB here)
    assert 14 * 4096 * 300 < b - a < 14 * 4096 * 300 + 200_000


def test_workspace_size_scales_with_capacity():
    import paper_1610_01071_amd.efpi as E
    a = E.efpi_workspace_size(E.ConfigSpec([E.ReplicaSpec(4096, 4096.0, ppc=1000)]).to_c())
    b = E.efpi_workspace_size(E.ConfigSpec([E.ReplicaSpec(4096, 4096.0, ppc=2000)]).to_c())
    # 14 bytes per particle slot (int16 cell + 3 x FP32)
    assert abs((b - a) - 14 * 4096 * 1000) < 4096
    c = E.efpi_workspace_size(E.ConfigSpec([E.ReplicaSpec(4096, 4096.0, ppc=1000)],
                                           flags=E.FLAG_SORT_BUFFER).to_c())
    assert c > a + 14 * 4096 * 1000


def test_autotune_cache_roundtrip(tmp_path):
    """Cache keys and files of the autotuner (host only)."""
    from paper_1610_01071_amd import autotune
    import paper_1610_01071_amd.efpi as E
    specs = [E.ReplicaSpec(256, 256.0, ppc=10), E.ReplicaSpec(1024, 1024.0, ppc=20, bc=1)]
    k = autotune.cache_key(specs)
    assert "256x10x20x0" in k and "1024x20x20x1" in k
    path = str(tmp_path / "sub" / "t.json")
    autotune.save_cache(path, {k: {"tile": 2048, "grid_blocks": 4096, "ms_per_step": 1.0}})
    assert autotune.load_cache(path)[k]["tile"] == 2048
    assert autotune.load_cache(str(tmp_path / "missing.json")) == {}


def test_next_macro_dt_against_the_oracles_rule():
    """The library's step-size rule (host code) against the oracle's, written apart:
    the same steps over errors from 0 to far above tol, at and inside the clamps."""
    from oracle import efpi as oefpi
    import paper_1610_01071_amd.efpi as E
    for dt in (2.0, 5.0, 7.5):
        for err in (0.0, 1e-9, 1e-5, 2.5e-4, 1e-3, 4e-3, 1e-2, 1.0):
            for tol, lo, hi, safety in ((1e-3, 2.0, 40.0, 0.9), (3e-4, 5.0, 7.5, 1.0)):
                got = E.efpi_next_macro_dt(dt, err, tol, lo, hi, safety)
                assert got == oefpi.next_macro_dt(dt, err, tol, lo, hi, safety)
    for bad in ((0.0, 0.0, 1e-3, 1.0, 2.0), (1.0, -1.0, 1e-3, 1.0, 2.0), (1.0, 0.0, 0.0, 1.0, 2.0),
                (1.0, 0.0, 1e-3, 3.0, 2.0), (1.0, float("nan"), 1e-3, 1.0, 2.0)):
        with pytest.raises(E.EfpiError):
            E.efpi_next_macro_dt(*bad)
