"""The launch-shape autotuner: the tuned standalone form and lane count are
one of the product's own instantiations, so a product after tuning equals,
bitwise, the product forced to that form and lane count; other index arrays
keep the built-in rule (vector rows, lane rule)."""

import os

import numpy as np
import pytest
import torch

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hz():
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    import paper_2112_06465_amd as hz

    return hz


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def forced(hz, L, *args, form=None):
    os.environ["HZ_SPMV_LANES"] = str(L)
    if form is not None:
        os.environ["HZ_SPMV_FORM"] = form
    try:
        return hz.csr_zspmv(*args).cpu().numpy()
    finally:
        del os.environ["HZ_SPMV_LANES"]
        os.environ.pop("HZ_SPMV_FORM", None)


def test_tuned_lanes_are_used_bitwise_and_only_for_that_matrix(hz):
    A, b, _ = W.config_cube(30, seed=1)
    rp, ci, v = dev(A.row_ptr), dev(A.col_idx), dev(A.vals)
    x = dev(np.random.default_rng(3).standard_normal(A.n) + 1j * np.random.default_rng(4).standard_normal(A.n))
    os.environ.pop("HZ_SPMV_LANES", None)
    rule = hz.csr_zspmv(rp.clone(), ci.clone(), v, x).cpu().numpy()  # fresh index arrays: never tuned
    tune = hz.autotune_spmv(rp, ci, v, x, details=True)
    assert tune["lanes"] in (1, 2, 4, 8, 16, 32, 64) and tune["form_lanes"] in (2, 4, 8, 16, 32, 64)
    assert tune["form"] in ("rows", "tiles")
    y = hz.csr_zspmv(rp, ci, v, x).cpu().numpy()
    yf = forced(hz, tune["form_lanes"], rp, ci, v, x, form=tune["form"])
    assert np.array_equal(y.view(np.float64), yf.view(np.float64))
    yo = O.zspmv(A, x.cpu().numpy())
    assert np.linalg.norm(y - yo) / np.linalg.norm(yo) <= 1e-14
    # copies of the index arrays are another matrix for the handle: the rule applies
    mean = A.nnz / A.n
    Lr = 2
    while Lr < 64 and 2 * Lr < mean:
        Lr *= 2
    r2 = hz.csr_zspmv(rp.clone(), ci.clone(), v, x).cpu().numpy()
    assert np.array_equal(r2.view(np.float64), rule.view(np.float64))
    # untuned: block tiles for rows of at most 16 entries on average, else vector rows with the lane rule
    untuned = "tiles" if mean <= 16 else "rows"
    assert np.array_equal(rule.view(np.float64), forced(hz, Lr, rp, ci, v, x, form=untuned).view(np.float64))
    # a solve on the tuned matrix still meets its tolerance
    xs, info = hz.zbicgstab_solve(rp, ci, v, dev(b), rtol=1e-9)
    assert info["status"] == hz.OK
    xs = xs.cpu().numpy()
    assert np.linalg.norm(b - O.zspmv(A, xs)) / np.linalg.norm(b) <= 1e-9 * (1 + 1e-3)


def test_every_forced_lane_count_matches_the_oracle(hz):
    A, _, _ = W.config_cube(14, seed=2)
    rp, ci, v = dev(A.row_ptr), dev(A.col_idx), dev(A.vals)
    xh = np.random.default_rng(5).standard_normal(A.n) + 1j * np.random.default_rng(6).standard_normal(A.n)
    yo = O.zspmv(A, xh)
    for L in (2, 4, 8, 16, 32, 64):
        y = forced(hz, L, rp, ci, v, dev(xh), form="rows")
        assert np.linalg.norm(y - yo) / np.linalg.norm(yo) <= 1e-14, L
    y = forced(hz, 4, rp, ci, v, dev(xh), form="tiles")
    assert np.linalg.norm(y - yo) / np.linalg.norm(yo) <= 1e-14


def test_autotune_of_an_empty_matrix_and_return_forms(hz):
    rp = dev(np.zeros(4, np.int32))
    ci = dev(np.zeros(0, np.int32))
    v = dev(np.zeros(0, complex))
    tune = hz.autotune_spmv(rp, ci, v, dev(np.ones(3, complex)), details=True)
    assert tune["form"] == "rows"
    assert np.array_equal(hz.csr_zspmv(rp, ci, v, dev(np.ones(3, complex))).cpu().numpy(), np.zeros(3))


def test_tuning_cache_records_and_reuses_choices(hz, tmp_path):
    """A JSON tuning cache keyed by the matrix's shape: the first call times and stores, a call for other index
    arrays of the same shape records the stored choice without timing, and that choice is the one used."""
    import json

    A, _, _ = W.config_cube(24, seed=3)
    rp, ci, v = dev(A.row_ptr), dev(A.col_idx), dev(A.vals)
    x = dev(np.random.default_rng(2).standard_normal(A.n) + 0j)
    path = str(tmp_path / "tune.json")
    t1 = hz.autotune_spmv(rp, ci, v, x, details=True, cache=path)
    assert t1["cached"] is False
    stored = json.load(open(path))
    assert len(stored) == 1
    (entry,) = stored.values()
    assert entry == {k: t1[k] for k in ("lanes", "form", "form_lanes")}
    rp2, ci2 = rp.clone(), ci.clone()
    t2 = hz.autotune_spmv(rp2, ci2, v, x, details=True, cache=path)
    assert t2["cached"] is True and {k: t2[k] for k in entry} == entry
    y = hz.csr_zspmv(rp2, ci2, v, x).cpu().numpy()
    yf = forced(hz, t2["form_lanes"], rp2, ci2, v, x, form=t2["form"])
    assert np.array_equal(y.view(np.float64), yf.view(np.float64))
    L = hz.load()
    h = hz.handle(torch.device("cuda:0"))
    for lanes, form, fl in ((3, 0, 8), (8, 0, 5), (8, 1, 8), (8, 2, 8)):
        assert L.hz_autotune_set(h, A.n, A.nnz, rp2.data_ptr(), ci2.data_ptr(), lanes, form, fl) == -1
