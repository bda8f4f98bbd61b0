"""CPU checks of the C-ABI library: it loads, exports every symbol the header
declares, validates arguments, and its host-only partition is bit-identical
to the oracle's (no GPU needed: build_partition does no device work)."""
import os
import re

import numpy as np
import pytest

from oracle.partition import build_partition as oracle_partition
from paper_1104_3349_amd import addns
from workloads.configs import CAVITY16, CAVITY128, CAVITY256_STRETCHED
from workloads.mac_oseen import Wind, make_oseen_mac

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "addns.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(addns_[a-z_]+)\s*\(", src)))


def test_exports_every_declared_symbol():
    L = addns.lib()
    names = _declared()
    assert len(names) >= 13
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(addns.EXPORTED)
    assert addns.version().startswith("libaddns")


def _same(P, A):
    return all([np.array_equal(P.perm, A.perm), np.array_equal(P.part, A.part),
                np.array_equal(P.int_offsets, A.int_offsets),
                np.array_equal(P.agg_offsets, A.agg_offsets),
                np.array_equal(P.drange_offsets, A.drange_offsets),
                np.array_equal(P.drange_nodes, A.drange_nodes), np.array_equal(P.pair, A.pair),
                P.status == A.status])


@pytest.mark.parametrize("cfg", [CAVITY16, CAVITY128, CAVITY256_STRETCHED], ids=["cavity16", "cavity128", "cavity256s"])
def test_partition_bit_exact_configs(cfg):
    rp, ci, v, b, meta = cfg.build()
    P = oracle_partition(meta["N"], rp, ci, v, cfg.m, cfg.sz)
    A = addns.build_partition(meta["N"], rp, ci, v, cfg.m, cfg.sz).export()
    assert _same(P, A)


def test_partition_bit_exact_random():
    rng = np.random.default_rng(123)
    for _ in range(30):
        n = int(rng.integers(2, 34))
        st = [None, 1.03, 1.1][int(rng.integers(3))] if n % 2 == 0 else None
        w = Wind.random_modes(rng)
        rp, ci, v, b, meta = make_oseen_mac(n, float(rng.uniform(0.001, 0.3)), wind=w, stretch=st, seed=2)
        m, sz = int(rng.integers(1, 13)), int(rng.integers(1, 80))
        P = oracle_partition(meta["N"], rp, ci, v, m, sz)
        A = addns.build_partition(meta["N"], rp, ci, v, m, sz).export()
        assert _same(P, A), (n, m, sz)


def test_partition_argument_errors():
    rp, ci, v, b, meta = make_oseen_mac(6, 0.1, seed=1)
    with pytest.raises(addns.AddnsError) as e:
        addns.build_partition(meta["N"], rp, ci, v, 0, 8)
    assert e.value.code == addns.ERR_ARG and "m >= 1" in str(e.value)
    bad = ci.copy()
    bad[3] = meta["N"] + 5
    with pytest.raises(addns.AddnsError) as e:
        addns.build_partition(meta["N"], rp, bad, v, 2, 8)
    assert "out of range" in str(e.value)
    bad_rp = rp.copy()
    bad_rp[2], bad_rp[3] = bad_rp[3], bad_rp[2]
    with pytest.raises(addns.AddnsError):
        addns.build_partition(meta["N"], bad_rp, ci, v, 2, 8)


def test_partition_info_consistent():
    rp, ci, v, b, meta = make_oseen_mac(20, 0.02, seed=1)
    p = addns.build_partition(meta["N"], rp, ci, v, 5, 16)
    inf = p.info()
    A = p.export()
    assert inf["N"] == meta["N"] and inf["m"] == 5
    assert inf["n_interior"] + inf["sep_size"] == meta["N"]
    assert A.int_offsets[-1] == inf["n_interior"] and A.agg_offsets[-1] == inf["sep_size"]


def test_dtn_weights_file_roundtrip(tmp_path):
    """Host-only weight file I/O of the learned correction (no device work)."""
    n = addns.dtn_param_count()
    assert n == 4997
    w = np.random.default_rng(0).standard_normal(n).astype(np.float32)
    path = str(tmp_path / "dtn.bin")
    addns.dtn_save(path, w)
    assert os.path.getsize(path) == 8 + 4 + 4 * n
    assert np.array_equal(addns.dtn_load(path), w)
    with open(path, "r+b") as f:
        f.write(b"X")
    with pytest.raises(addns.AddnsError) as e:
        addns.dtn_load(path)
    assert e.value.code == addns.ERR_ARG
    with pytest.raises(addns.AddnsError):
        addns.dtn_load(str(tmp_path / "missing.bin"))


def _same_coarse(rp, ci, v, meta, m, sz, piece):
    from oracle.coarse import coarse_space
    P = oracle_partition(meta["N"], rp, ci, v, m, sz)
    offs, pos, zcols = coarse_space(meta["N"], rp, ci, P, piece)
    A = addns.build_partition(meta["N"], rp, ci, v, m, sz).coarse_space(piece)
    assert np.array_equal(A["piece_offsets"], offs)
    assert np.array_equal(A["piece_pos"], pos)
    assert np.array_equal(A["col_piece"], [c for c, _ in zcols])
    kinds, z0, z1 = [], np.zeros(P.sep_size), np.zeros(P.sep_size)
    last = -1
    for c, val in zcols:
        kinds.append(0 if c != last else 1)
        (z0 if c != last else z1)[pos[offs[c]:offs[c + 1]]] = val
        last = c
    assert np.array_equal(A["col_kind"], kinds)
    np.testing.assert_allclose(A["z0"], z0, rtol=0, atol=4e-16)
    np.testing.assert_allclose(A["z1"], z1, rtol=0, atol=4e-16)


@pytest.mark.parametrize("cfg", [CAVITY16, CAVITY128], ids=["cavity16", "cavity128"])
def test_coarse_space_matches_oracle_configs(cfg):
    rp, ci, v, b, meta = cfg.build()
    _same_coarse(rp, ci, v, meta, cfg.m, cfg.sz, 32)


def test_coarse_space_matches_oracle_random():
    rng = np.random.default_rng(321)
    for _ in range(12):
        n = int(rng.integers(4, 30))
        st = [None, 1.05][int(rng.integers(2))] if n % 2 == 0 else None
        rp, ci, v, b, meta = make_oseen_mac(n, float(rng.uniform(0.001, 0.3)), wind=Wind.random_modes(rng),
                                            stretch=st, seed=3)
        _same_coarse(rp, ci, v, meta, int(rng.integers(1, 9)), int(rng.integers(4, 70)),
                     int(rng.integers(1, 65)))


def test_coarse_space_argument_errors():
    rp, ci, v, b, meta = make_oseen_mac(6, 0.1, seed=1)
    p = addns.build_partition(meta["N"], rp, ci, v, 2, 8)
    for bad in (0, 65):
        with pytest.raises(addns.AddnsError) as e:
            p.coarse_space(bad)
        assert e.value.code == addns.ERR_ARG
