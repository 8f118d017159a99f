import hashlib
import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")


def _oracle_tables(**params):
    """Oracle look-up tables, cached on disk per (oracle source, parameters)."""
    import oracle
    p = dict(oracle.DEFAULT_TABLE_PARAMS)
    p.update(params)
    src = open(os.path.join(ROOT, "oracle", "qed_oracle.cpp"), "rb").read()
    key = hashlib.sha1(src + repr(sorted(p.items())).encode()).hexdigest()[:16]
    cache_dir = os.path.join(ROOT, "oracle", "_cache")
    path = os.path.join(cache_dir, "tables_%s.npz" % key)
    if os.path.exists(path):
        d = dict(np.load(path))
        d["params"] = p
        return d
    t = oracle.build_tables(**p)
    os.makedirs(cache_dir, exist_ok=True)
    tmp = path + ".tmp%d.npz" % os.getpid()
    np.savez(tmp, **{k: v for k, v in t.items() if k != "params"})
    os.replace(tmp, path)
    return t


@pytest.fixture(scope="session")
def oracle_tables():
    """Full-size tables (256 x 256, eta in [1e-4, 1e2], chi_pair in [1e-2, 1e2])."""
    return _oracle_tables()


@pytest.fixture(scope="session")
def oracle_tables_small():
    """Small tables for fast CPU tests (same ranges, 48-point grids)."""
    return _oracle_tables(n_eta=48, n_chi=48, n_chi_pair=48, n_f=48)


def pytest_collection_modifyitems(config, items):
    """GPU tests run where a GPU is visible; elsewhere they are skipped (never faked)."""
    if not any("gpu" in it.keywords for it in items):
        return
    try:
        import torch
        has_gpu = torch.cuda.is_available()
    except Exception:
        has_gpu = False
    if has_gpu:
        return
    skip = pytest.mark.skip(reason="no GPU visible")
    for it in items:
        if "gpu" in it.keywords:
            it.add_marker(skip)
