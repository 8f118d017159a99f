"""qed_sort_static (the entry point that allocates nothing) against qed_sort, through the C ABI:
two calls in a row on the same GPU, the second with a smaller input, each compared with
qed_sort on a twin run.  The order of particles inside a tile is not specified (it follows the
atomics), so what is compared is what is unique: every particle per uid, bit for bit, the tile
order of the slots, and the particles after further steps."""
import numpy as np
import pytest

from paper_1311_5551_amd import capi, workloads as W
from paper_1311_5551_amd.sim import Run, Tables

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def shared_tables(oracle_tables):
    return Tables.from_arrays(oracle_tables)


def _grid_run(tables, n, seed):
    w = W.grid_config3(n=n, nx=256, ny=64, n_steps=200, seed=seed)
    w.capacity = dict(electron=20 * w.n, positron=20 * w.n, photon=100 * w.n)
    return w, Run(w, tables)


def _by_uid(run, name):
    d = run.species(0, name, live_only=False)
    o = np.argsort(d["uid"])
    return {k: v[o] for k, v in d.items()}


def _tiles(run, w):
    e = run.species(0, "electron", live_only=False)
    nx, ny, dx, dy, x0, y0 = w.grid
    i = np.floor((e["x"] - x0) / dx).astype(np.int64) % nx
    j = np.floor((e["y"] - y0) / dy).astype(np.int64) % ny
    return (j // 8) * ((nx + 7) // 8) + i // 8


def _compare(ra, rb):
    for name in ("electron", "positron", "photon"):
        a, b = _by_uid(ra, name), _by_uid(rb, name)
        assert len(a["uid"]) == len(b["uid"]), name
        for k in a:
            np.testing.assert_array_equal(a[k], b[k], err_msg="%s.%s" % (name, k))


@pytest.mark.parametrize("n,seed", [(3000, 2), (900, 5)])
def test_sort_static_equals_sort(n, seed, shared_tables):
    # the second case runs after the first in the same process: a smaller input on the same array
    w, ra = _grid_run(shared_tables, n, seed)
    _, rb = _grid_run(shared_tables, n, seed)
    ra.step(60)
    rb.step(60)
    ra.sort()
    rb.sort_static()
    _compare(ra, rb)
    assert np.all(np.diff(_tiles(rb, w)) >= 0)  # slots in tile order
    for _ in range(5):
        ra.step(10)
        rb.step(10)
        ra.sort()
        rb.sort_static()
    _compare(ra, rb)
    la, lb = ra.ledger()[0], rb.ledger()[0]
    assert la["status"] == lb["status"] == "QED_OK"
    assert (la["n_emit"], la["n_pair"]) == (lb["n_emit"], lb["n_pair"])


def test_sort_static_rejects_species_beyond_its_scratch(shared_tables):
    w = W.grid_config3(n=1000, nx=256, ny=64, n_steps=10, seed=3)
    w.capacity = dict(electron=(1 << 21) + 1, positron=1024, photon=1024)
    r = Run(w, shared_tables)
    with pytest.raises(capi.QEDError) as e:
        r.sort_static()
    assert e.value.status == capi.QED_ERR_ARG
    assert b"2097152" in capi.lib().qed_last_error()
    r.step(2)  # nothing was enqueued; the run goes on
    assert r.ledger()[0]["status"] == "QED_OK"
