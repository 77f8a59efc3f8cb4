"""The one-launch reductions zdotc and dznrm2: slots, fixed order, bounded wait.

Each block publishes its total in a slot of the handle and the grid's last
block adds the slots in index order.  Checked here: results against the
oracle at a size where blocks take several chunks each; bitwise equality of
repeated calls when calls of different sizes (and so different block counts)
alternate on one handle, eagerly and as replays of a captured graph; and the
failure path of the bounded wait, forced from the host with a wait limit of
0 ticks on a handle of its own, which must write NaN and keep writing NaN on
that handle while the default handle stays correct.
"""

import ctypes as C
import os

import numpy as np
import pytest
import torch

import oracle as O

pytestmark = pytest.mark.gpu

EPS = np.finfo(float).eps
SIZES = [0, 1, 1000, 209_777, 3_000_001]  # 3,000,001 elements: 2 chunks per block over 1,465 blocks


@pytest.fixture(scope="module")
def hz():
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    import paper_2112_06465_amd as hz

    return hz


def cn(rng, n):
    return rng.standard_normal(n) + 1j * rng.standard_normal(n)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def test_multi_chunk_blocks_against_the_oracle(hz):
    n = SIZES[-1]
    rng = np.random.default_rng(11)
    x, y = cn(rng, n), cn(rng, n)
    d = complex(hz.zdotc(dev(x), dev(y)).cpu())
    scale = np.sum(np.abs(x) * np.abs(y))
    assert abs(d - O.zdotc(x, y)) <= n * EPS * scale
    nr = float(hz.dznrm2(dev(x)).cpu())
    assert abs(nr - O.dznrm2(x)) <= n * EPS * O.dznrm2(x)


def test_alternating_sizes_repeat_bitwise(hz):
    rng = np.random.default_rng(5)
    vecs = [(dev(cn(rng, n)), dev(cn(rng, n))) for n in SIZES]
    first = [(hz.zdotc(x, y).clone(), hz.dznrm2(x).clone()) for x, y in vecs]
    assert complex(first[0][0].cpu()) == 0 and float(first[0][1].cpu()) == 0.0
    for rnd in range(3):
        order = range(len(SIZES)) if rnd % 2 == 0 else reversed(range(len(SIZES)))
        for i in order:
            x, y = vecs[i]
            assert torch.equal(hz.zdotc(x, y), first[i][0]), (rnd, SIZES[i])
            assert torch.equal(hz.dznrm2(x), first[i][1]), (rnd, SIZES[i])


def test_graph_replays_match_eager_calls(hz):
    rng = np.random.default_rng(6)
    vecs = [(dev(cn(rng, n)), dev(cn(rng, n))) for n in SIZES[1:]]
    eager = [(hz.zdotc(x, y).clone(), hz.dznrm2(y).clone()) for x, y in vecs]
    outs = [(torch.empty((), dtype=torch.complex128, device="cuda:0"),
             torch.empty((), dtype=torch.float64, device="cuda:0")) for _ in vecs]
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):  # warm-up on the capture stream
        for (x, y), (od, on) in zip(vecs, outs):
            od.copy_(hz.zdotc(x, y))
    torch.cuda.current_stream().wait_stream(s)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        for _ in range(3):
            for (x, y), (od, on) in zip(vecs, outs):
                hz.zdotc(x, y, out=od)
                hz.dznrm2(y, out=on)
    for rep in range(4):
        for od, on in outs:
            od.fill_(float("nan"))
            on.fill_(float("nan"))
        g.replay()
        torch.cuda.synchronize()
        for i, (od, on) in enumerate(outs):
            assert torch.equal(od, eager[i][0]), (rep, i)
            assert torch.equal(on, eager[i][1]), (rep, i)
        # eager calls of other sizes between replays
        x, y = vecs[rep % len(vecs)]
        assert torch.equal(hz.zdotc(x, y), eager[rep % len(vecs)][0])


def test_wait_that_gives_up_writes_nan_and_poisons_only_its_handle(hz):
    from paper_2112_06465_amd._lib import load

    L = load()
    os.environ["HZ_B1_WAIT_TICKS"] = "0"
    try:
        hp = C.c_void_p()
        assert L.hz_handle_create(C.byref(hp)) == 0
    finally:
        del os.environ["HZ_B1_WAIT_TICKS"]
    h = hp.value
    try:
        rng = np.random.default_rng(8)
        n = 209_777
        x, y = dev(cn(rng, n)), dev(cn(rng, n))
        od = torch.zeros((), dtype=torch.complex128, device="cuda:0")
        on = torch.zeros((), dtype=torch.float64, device="cuda:0")
        st = torch.cuda.current_stream().cuda_stream
        for _ in range(2):
            assert L.zdotc(h, st, n, x.data_ptr(), y.data_ptr(), od.data_ptr()) == 0
            assert L.dznrm2(h, st, n, x.data_ptr(), on.data_ptr()) == 0
            torch.cuda.synchronize()
            assert np.isnan(complex(od.cpu()).real) and np.isnan(float(on.cpu()))
        # the default handle is untouched
        ref = O.zdotc(x.cpu().numpy(), y.cpu().numpy())
        d = complex(hz.zdotc(x, y).cpu())
        assert abs(d - ref) <= n * EPS * float((x.abs() * y.abs()).sum())
    finally:
        L.hz_handle_destroy(C.c_void_p(h))
