"""crk_workspace_estimate (host only): the up-front bound grows with the
particle and pair counts, every extra use adds to it, and bad arguments are
refused. (The GPU test bounds a real step's workspace by it.)"""
import pytest

from paper_2202_02840_amd import _lib
from paper_2202_02840_amd._lib import (CRK_FP64, CRK_MIXED, CRK_MIXED_ADAPT, WS_COMPAT, WS_GRAPH,
                                       WS_HNET, WS_HSOLVE, WS_LEAVES, WS_TIMESTEP, WS_VERLET,
                                       CrkError, workspace_estimate)


def test_monotone_in_size_and_pairs():
    a = workspace_estimate(1 << 15, 64.0, CRK_MIXED_ADAPT)
    b = workspace_estimate(1 << 18, 64.0, CRK_MIXED_ADAPT)
    c = workspace_estimate(1 << 18, 128.0, CRK_MIXED_ADAPT)
    assert a < b < c
    # at least the sorted positions, records and the pair lists
    n, ppp = 1 << 18, 128.0
    assert c >= n * (32 + 144 + 16) + 4 * n * ppp


def test_each_use_adds():
    base = workspace_estimate(100000, 80.0, CRK_MIXED_ADAPT)
    for u in (WS_HSOLVE, WS_HNET, WS_COMPAT, WS_VERLET, WS_GRAPH, WS_TIMESTEP, WS_LEAVES):
        assert workspace_estimate(100000, 80.0, CRK_MIXED_ADAPT, u) > base, u


def test_fp64_records_are_larger():
    assert workspace_estimate(100000, 80.0, CRK_FP64) > workspace_estimate(100000, 80.0, CRK_MIXED)


@pytest.mark.parametrize("args", [(0, 80.0, 0), (10, -1.0, 0), (10, 80.0, 7)])
def test_bad_arguments(args):
    with pytest.raises(CrkError):
        workspace_estimate(*args)


def test_full_size_fits_one_gpu():
    # 256^3 clustered, about 90 pairs per particle, whole step with the h
    # iteration and the network: well inside 288 GB of HBM
    b = workspace_estimate(256 ** 3, 90.0, CRK_MIXED_ADAPT, WS_HSOLVE | WS_HNET)
    assert 1e10 < b < 2.0e11
