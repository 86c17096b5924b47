"""The C ABI: every declared entry point is exported, and host-side validation
works without a GPU."""
import ctypes
import os
import re

import pytest

from paper_1208_0274_amd import alae

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "alae.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z_0-9]*\s*\*?\s*(alae_[a-z_0-9]+)\s*\(", src, flags=re.M)
    return sorted(set(names))


def test_every_declared_symbol_is_exported():
    names = declared_functions()
    assert len(names) >= 15
    lib = ctypes.CDLL(alae.LIB_PATH)
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_version():
    assert "gfx950" in alae.version()


@pytest.mark.parametrize("kw,status", [
    (dict(sa=0, sb=-3, sg=-5, ss=-2), 3),
    (dict(sa=1, sb=1, sg=-5, ss=-2), 3),
    (dict(sa=1, sb=-3, sg=1, ss=-2), 3),
    (dict(sa=1, sb=-3, sg=-5, ss=0), 3),
])
def test_scoring_validation(kw, status):
    idx = alae.Index.build("ACGTACGTTTGACA", "dna")
    with pytest.raises(alae.AlaeError) as ei:
        alae.search(idx, "ACGT", 3, alae.make_scoring(**kw))
    assert ei.value.status == status


def test_query_validation():
    idx = alae.Index.build("ACGTACGTTTGACA", "dna")
    with pytest.raises(alae.AlaeError) as ei:
        alae.search(idx, "ACXT", 3)
    assert ei.value.status == 2
    with pytest.raises(alae.AlaeError) as ei:
        alae.search(idx, "ACGT", 0)
    assert ei.value.status == 3
    with pytest.raises(alae.AlaeError) as ei:
        alae.search(idx, "", 3)
    assert ei.value.status == 1
    m = [[1, 2, 0, 0], [0, 1, 0, 0], [0, 0, 1, 0], [0, 0, 0, 1]]  # asymmetric
    with pytest.raises(alae.AlaeError) as ei:
        alae.search(idx, "ACGT", 3, alae.make_scoring(matrix=m))
    assert ei.value.status == 3


@pytest.mark.parametrize("shape", [dict(level_stage=3), dict(level_stage=16), dict(wide_blocks_per_cu=9),
                                   dict(lane_waves_per_cu=17), dict(wide_blocks_per_cu=-1)])
def test_launch_shape_validation(shape):
    """Unsupported launch shapes are rejected before any device work."""
    idx = alae.Index.build("ACGTACGTTTGACA", "dna")
    with pytest.raises(alae.AlaeError) as ei:
        alae.search(idx, "ACGT", 3, **shape)
    assert ei.value.status == 1
