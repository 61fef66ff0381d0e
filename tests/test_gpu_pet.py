"""GPU parity of the penalized PET reconstruction MM algorithm (Sec. 3.2,
Algorithm 2) against the float64 oracle oracle/pet_oracle.py, on the same
float32 inputs, through the C ABI (nmf_pet_*).

Workloads: the 64 x 64 image seen by 2016 lines of flight of a 64-detector
ring (the paper's problem size, synthetic geometry and phantom), and a small
ragged problem (37 lines, 9 x 12 grid, a pixel that no line crosses, lines
with zero counts) that exercises the padding and the b > 0 branch of the
root.

Bars (float32 products against float64): f within 1e-5 relative at each of
the first 20 iterations and lambda within 1e-4 relative (Frobenius) after
20; f non-decreasing (float32 slack 1e-6 |f|); bit-identical intensities for
every split of the iterations over the replayed graphs."""
import numpy as np
import pytest
import torch

from oracle import pet_oracle as O
from synth import generators as g

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def full_problem():
    E, y, _ = g.pet_problem()
    return E, y, 64, 64


def _ragged_problem():
    rng = np.random.default_rng(6100)
    rows, cols, d = 9, 12, 37
    p = rows * cols
    E = rng.exponential(1.0, size=(d, p)) * (rng.uniform(size=(d, p)) < 0.2)
    E[:, 50] = 0.0                                   # a pixel no line crosses
    lam_true = rng.gamma(2.0, 2.0, size=p)
    y = rng.poisson(E @ lam_true).astype(np.float64)
    y[::5] = 0.0                                     # lines with zero counts
    return E.astype(np.float32), y.astype(np.float32), rows, cols


def rel(a, b):
    a = np.asarray(a, np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _gpu_run(E, y, rows, cols, mu, iters, lam0=None, each=True, layout="auto", expect=None):
    from paper_1003_3272_amd import nmf
    p = E.shape[1]
    lam0 = np.ones(p, np.float32) if lam0 is None else lam0
    Ed, yd, ld = (torch.from_numpy(np.ascontiguousarray(x)).cuda() for x in (E, y, lam0))
    trace = []
    with nmf.Pet(Ed, yd, ld, rows, cols, mu, layout=layout) as m:
        if expect is not None:
            assert m.layout == expect
        trace.append(m.objective())
        if each:
            for _ in range(iters):
                m.step(1)
                trace.append(m.objective())
        else:
            m.step(iters)
            trace.append(m.objective())
    return ld.cpu().numpy(), np.array(trace)


# the ring geometry is about 2% dense: AUTO takes the sparse layout
@pytest.mark.parametrize("layout,expect", [("auto", "sparse"), ("dense", "dense")])
@pytest.mark.parametrize("mu", [0.0, 1e-5, 1e-3, 1e-1])
def test_pet_matches_oracle_full_size(gpu_lib, full_problem, mu, layout, expect):
    E, y, rows, cols = full_problem
    pairs = O.neighbour_pairs(rows, cols)
    lam, tr = _gpu_run(E, y, rows, cols, mu, 20, layout=layout, expect=expect)
    lam_o, tr_o = O.run(E, y, np.ones(E.shape[1]), mu, pairs, 20)
    err = np.abs(tr - tr_o) / np.abs(tr_o)
    assert err.max() < 1e-5, (mu, err.max(), int(err.argmax()))
    assert rel(lam, lam_o) < 1e-4
    assert (lam >= 0).all()


# 20% dense: AUTO keeps the dense layout
@pytest.mark.parametrize("layout,expect", [("auto", "dense"), ("sparse", "sparse")])
@pytest.mark.parametrize("mu", [0.0, 1e-2, 1.0])
def test_pet_matches_oracle_ragged(gpu_lib, mu, layout, expect):
    E, y, rows, cols = _ragged_problem()
    pairs = O.neighbour_pairs(rows, cols)
    lam, tr = _gpu_run(E, y, rows, cols, mu, 20, layout=layout, expect=expect)
    lam_o, tr_o = O.run(E, y, np.ones(E.shape[1]), mu, pairs, 20)
    err = np.abs(tr - tr_o) / np.maximum(np.abs(tr_o), 1.0)
    assert err.max() < 1e-5, (mu, err.max())
    assert rel(lam, lam_o) < 1e-4
    # the uncrossed pixel has c = 0: it is 0 while b <= 0 and -b / a once
    # its neighbours make b positive (at mu = 1, from the first iteration)
    assert abs(lam[50] - lam_o[50]) <= 1e-4 * lam_o.max()
    if mu >= 1.0:
        assert lam_o[50] > 0
    if mu == 0.0:
        assert lam[50] == 0.0


def test_pet_matches_oracle_many_lines_per_pixel(gpu_lib):
    """301 lines over an 8 x 8 grid, 25% dense: more than 32 lines cross a
    pixel, so the sparse update takes a whole wave per pixel."""
    rng = np.random.default_rng(6102)
    d, rows, cols = 301, 8, 8
    E = (rng.uniform(0.1, 1.0, size=(d, rows * cols)) *
         (rng.uniform(size=(d, rows * cols)) < 0.25)).astype(np.float32)
    y = rng.poisson(E @ rng.gamma(2.0, 2.0, size=rows * cols)).astype(np.float32)
    pairs = O.neighbour_pairs(rows, cols)
    lam_o, tr_o = O.run(E, y, np.ones(rows * cols), 0.05, pairs, 20)
    for layout in ("sparse", "dense"):
        lam, tr = _gpu_run(E, y, rows, cols, 0.05, 20, layout=layout, expect=layout)
        assert (np.abs(tr - tr_o) / np.abs(tr_o)).max() < 1e-5
        assert rel(lam, lam_o) < 1e-4


def test_pet_tiny_penalty_root_is_stable(gpu_lib, full_problem):
    """At mu = 1e-9 the printed root form cancels in float32; the kernel's
    form must still track the float64 oracle (whose own cancellation costs
    about 1e-9 relative here)."""
    E, y, rows, cols = full_problem
    pairs = O.neighbour_pairs(rows, cols)
    lam, _ = _gpu_run(E, y, rows, cols, 1e-9, 5, each=False)
    lam_o, _ = O.run(E, y, np.ones(E.shape[1]), 1e-9, pairs, 5)
    assert rel(lam, lam_o) < 1e-5


@pytest.mark.parametrize("mu", [0.0, 1e-3])
def test_pet_objective_ascends(gpu_lib, full_problem, mu):
    from paper_1003_3272_amd import nmf
    E, y, rows, cols = full_problem
    Ed, yd = torch.from_numpy(E).cuda(), torch.from_numpy(y).cuda()
    ld = torch.ones(E.shape[1], dtype=torch.float32, device="cuda")
    with nmf.Pet(Ed, yd, ld, rows, cols, mu) as m:
        fs = [m.objective()]
        for _ in range(40):
            m.step(7)
            fs.append(m.objective())
    fs = np.array(fs)
    slack = 1e-6 * np.abs(fs[1:])
    assert (np.diff(fs) >= -slack).all(), np.diff(fs).min()
    assert fs[-1] > fs[0]


@pytest.mark.parametrize("layout", ["sparse", "dense"])
def test_pet_graph_splits_are_bit_identical(gpu_lib, full_problem, layout):
    E, y, rows, cols = full_problem
    kw = dict(layout=layout)
    a, _ = _gpu_run(E, y, rows, cols, 1e-4, 23, each=False, **kw)      # 16 + 4 + 2 + 1
    b, _ = _gpu_run(E, y, rows, cols, 1e-4, 23, each=True, **kw)       # 23 x 1
    c, _ = _gpu_run(E, y, rows, cols, 1e-4, 23, each=False, **kw)
    assert np.array_equal(a, b) and np.array_equal(a, c)


def test_pet_layouts_agree(gpu_lib, full_problem):
    E, y, rows, cols = full_problem
    a, ta = _gpu_run(E, y, rows, cols, 1e-4, 50, each=False, layout="sparse")
    b, tb = _gpu_run(E, y, rows, cols, 1e-4, 50, each=False, layout="dense")
    assert rel(a, b) < 1e-5
    assert abs(ta[-1] - tb[-1]) <= 1e-7 * abs(tb[-1])


def test_pet_rejects_negative_or_nonfinite_data(gpu_lib):
    from paper_1003_3272_amd import nmf
    E, y, rows, cols = _ragged_problem()
    for what in ("E", "y", "lam"):
        Eb, yb, lb = E.copy(), y.copy(), np.ones(E.shape[1], np.float32)
        {"E": Eb, "y": yb, "lam": lb}[what].flat[3] = -1.0 if what != "y" else np.nan
        Ed, yd, ld = (torch.from_numpy(x).cuda() for x in (Eb, yb, lb))
        with pytest.raises(nmf.NmfError) as ei:
            nmf.Pet(Ed, yd, ld, rows, cols, 0.1)
        assert ei.value.status == nmf.NMF_EINVAL


def test_pet_solve_stopping_rule(gpu_lib, full_problem):
    from paper_1003_3272_amd import nmf
    E, y, rows, cols = full_problem
    pairs = O.neighbour_pairs(rows, cols)
    Ed, yd = torch.from_numpy(E).cuda(), torch.from_numpy(y).cuda()
    ld = torch.ones(E.shape[1], dtype=torch.float32, device="cuda")
    with nmf.Pet(Ed, yd, ld, rows, cols, 1e-2) as m:
        conv, it, f = m.solve(5, tol=0.0)
        assert not conv and it == 5
        conv, it, f = m.solve(20000, tol=1e-7, check_every=4)
        assert conv and 0 < it < 20000 and it % 4 == 0
        assert f == m.objective()
        f_next = (m.step(4), m.objective())[1]
        assert abs(f_next - f) / (abs(f) + 1.0) < 1e-6
    lam = ld.cpu().numpy()
    fo = O.objective(O.scale_columns(E), y, lam, 1e-2, pairs)
    assert abs(fo - f_next) <= 1e-6 * abs(fo)


def test_pet_start_is_the_callers(gpu_lib):
    """lambda is the caller's buffer: a non-uniform start is used as given
    and updated in place."""
    E, y, rows, cols = _ragged_problem()
    lam0 = np.random.default_rng(6101).uniform(0.5, 2.0, size=E.shape[1]).astype(np.float32)
    pairs = O.neighbour_pairs(rows, cols)
    lam, tr = _gpu_run(E, y, rows, cols, 1e-2, 3, lam0=lam0)
    lam_o, tr_o = O.run(E, y, lam0, 1e-2, pairs, 3)
    assert abs(tr[0] - tr_o[0]) <= 1e-6 * max(abs(tr_o[0]), 1.0)
    assert rel(lam, lam_o) < 1e-5


# ---- QN(q) acceleration (Table 3, QN(10) columns) -----------------------------

def test_pet_qn_first_iterations_match_oracle(gpu_lib, full_problem):
    """QN(10) from lambda = 1 at mu = 1e-5: the accepted objective after
    each of the first 6 QN iterations within 1e-6 relative of the float64
    oracle's (later iterations depend on ill-conditioned secant systems and
    are compared through their limit instead)."""
    from paper_1003_3272_amd import nmf
    E, y, rows, cols = full_problem
    pairs = O.neighbour_pairs(rows, cols)
    _, _, _, tr_o, acc_o = O.solve_qn(E, y, np.ones(E.shape[1]), 1e-5, pairs, 10, 12)
    Ed, yd = torch.from_numpy(E).cuda(), torch.from_numpy(y).cuda()
    ld = torch.ones(E.shape[1], dtype=torch.float32, device="cuda")
    with nmf.Pet(Ed, yd, ld, rows, cols, 1e-5) as m:
        conv, ev, acc, f, tr = m.solve_qn(12, q=10, tol=0.0, trace_len=7)
    assert ev == 12 and len(tr) == 7
    err = np.abs(np.array(tr) - tr_o[:7]) / np.abs(tr_o[:7])
    assert err.max() < 1e-6, err
    assert abs(acc - acc_o) <= 1


@pytest.mark.parametrize("mu", [1e-5, 1e-3])
def test_pet_qn_reaches_the_maximum_in_fewer_evaluations(gpu_lib, full_problem, mu):
    """To the stopping rule at 1e-10, QN(10) needs far fewer map evaluations
    than plain MM and ends at an objective no lower (f is concave, so both
    approach the same maximum; the slower MM stops further below it)."""
    from paper_1003_3272_amd import nmf
    E, y, rows, cols = full_problem
    Ed, yd = torch.from_numpy(E).cuda(), torch.from_numpy(y).cuda()
    res = {}
    for kind in ("mm", "qn"):
        ld = torch.ones(E.shape[1], dtype=torch.float32, device="cuda")
        with nmf.Pet(Ed, yd, ld, rows, cols, mu) as m:
            if kind == "mm":
                conv, it, f = m.solve(100000, tol=1e-10, check_every=1)
                res[kind] = (conv, it, f)
            else:
                conv, ev, acc, f, tr = m.solve_qn(100000, q=10, tol=1e-10, check_every=2,
                                                  trace_len=100001)
                res[kind] = (conv, ev, f)
                tr = np.array(tr)
                assert (np.diff(tr) >= -1e-6 * np.abs(tr[1:])).all()
                assert acc > 0
                assert f == m.objective()
    assert res["mm"][0] and res["qn"][0]
    assert res["qn"][1] < res["mm"][1] / 2, res
    assert res["qn"][2] >= res["mm"][2] - 1e-7 * abs(res["mm"][2]), res


def test_pet_qn_then_plain_steps_continue(gpu_lib):
    from paper_1003_3272_amd import nmf
    E, y, rows, cols = _ragged_problem()
    Ed, yd = torch.from_numpy(E).cuda(), torch.from_numpy(y).cuda()
    ld = torch.ones(E.shape[1], dtype=torch.float32, device="cuda")
    pairs = O.neighbour_pairs(rows, cols)
    with nmf.Pet(Ed, yd, ld, rows, cols, 1e-2) as m:
        conv, ev, acc, f, _ = m.solve_qn(40, q=4, tol=0.0)
        lam_after = ld.cpu().numpy()
        assert abs(O.objective(O.scale_columns(E), y, lam_after, 1e-2, pairs) - f) <= 1e-6 * abs(f)
        m.step(10)
        assert m.objective() >= f - 1e-6 * abs(f)
        for q in (0, 17):
            with pytest.raises(nmf.NmfError) as e:
                m.solve_qn(10, q=q)
            assert e.value.status == nmf.NMF_EINVAL


@pytest.mark.parametrize("check_every,max_iters", [(3, 500), (1, 40), (7, 45)])
def test_pet_solve_matches_a_host_loop(gpu_lib, full_problem, check_every, max_iters):
    """The solve tests the rule on the device between replayed blocks of
    iterations; a host loop of steps and objectives with the same rule must
    stop at the same iteration with the same f and intensities, bit for bit
    (including a last block shorter than check_every at the cap)."""
    from paper_1003_3272_amd import nmf
    E, y, rows, cols = full_problem
    Ed, yd = torch.from_numpy(E).cuda(), torch.from_numpy(y).cuda()
    la = torch.ones(E.shape[1], dtype=torch.float32, device="cuda")
    lb = torch.ones(E.shape[1], dtype=torch.float32, device="cuda")
    tol = 1e-7 if max_iters == 500 else 0.0
    with nmf.Pet(Ed, yd, la, rows, cols, 1e-3) as ma, nmf.Pet(Ed, yd, lb, rows, cols, 1e-3) as mb:
        conv, it, f = ma.solve(max_iters, tol=tol, check_every=check_every)
        f_prev, k, conv_b = mb.objective(), 0, False
        while k < max_iters:
            todo = min(check_every, max_iters - k)
            mb.step(todo)
            k += todo
            fb = mb.objective()
            if abs(fb - f_prev) / (abs(f_prev) + 1.0) < tol:
                conv_b = True
                break
            f_prev = fb
        assert (conv, it) == (conv_b, k)
        assert f == fb
    assert torch.equal(la, lb)
