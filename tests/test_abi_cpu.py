"""C-ABI checks that need no GPU: the library loads, exports every entry point
that include/nmf.h declares, and rejects bad arguments before any device
work."""
import ctypes
import os
import re

import pytest

from paper_1003_3272_amd import nmf

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    names = []
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if not fn.endswith(".h"):
            continue
        text = open(os.path.join(ROOT, "include", fn)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names += re.findall(r"\b(nmf_[a-z0-9_]+)\s*\(", text)
    return sorted(set(names))


def test_header_declares_entry_points():
    names = _declared_functions()
    for required in ("nmf_init", "nmf_step", "nmf_objective", "nmf_solve", "nmf_destroy"):
        assert required in names


def test_library_exports_every_declared_symbol():
    lib = nmf.load()
    missing = [n for n in _declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_options_struct_layout_matches_header():
    # int32, int32, double, int32, int32, uint64, int32, int32 -> 40 bytes
    assert ctypes.sizeof(nmf.NmfOptions) == 40
    assert nmf.NmfOptions.tol.offset == 8
    assert nmf.NmfOptions.seed.offset == 24
    assert nmf.NmfOptions.use_graph.offset == 32


def test_default_options():
    o = nmf.NmfOptions()
    nmf.load().nmf_default_options(ctypes.byref(o))
    assert (o.precision, o.tol_kind, o.tol, o.check_every, o.validate, o.seed,
            o.use_graph, o.loss) == (0, 0, 1e-9, 1, 0, 0, 1, 0)


def test_strerror_and_version():
    lib = nmf.load()
    for s in (0, 1, -1, -2, -3, -4, -5):
        assert len(nmf.strerror(s)) > 0
    assert nmf.strerror(99) == "unknown status"
    assert lib.nmf_version() >= 100


FAKE = 0x10000  # aligned, never dereferenced: checks reject before device work


def _init(V=FAKE, p=8, n=8, ldv=8, r=2, W=FAKE, H=FAKE, opt=None, out=True):
    lib = nmf.load()
    ctx = ctypes.c_void_p(123)
    o = opt if opt is not None else nmf.options()
    st = lib.nmf_init(ctypes.byref(ctx) if out else None, V, p, n, ldv, r, W, H,
                      ctypes.byref(o), None)
    return st, ctx


@pytest.mark.parametrize("kw", [
    dict(V=None), dict(W=None), dict(H=None), dict(p=0), dict(n=0), dict(r=0),
    dict(p=-3), dict(ldv=7), dict(V=FAKE + 2), dict(W=FAKE + 1), dict(H=FAKE + 3),
])
def test_init_rejects_bad_arguments(kw):
    st, ctx = _init(**kw)
    assert st == nmf.NMF_EINVAL
    assert ctx.value is None


def test_init_rejects_null_out():
    st, _ = _init(out=False)
    assert st == nmf.NMF_EINVAL


def test_init_rejects_rank_above_max():
    st, _ = _init(r=nmf.MAX_RANK + 1)
    assert st == nmf.NMF_EUNSUPPORTED


@pytest.mark.parametrize("field,value,code", [
    ("check_every", 0, nmf.NMF_EINVAL),
    ("tol", float("nan"), nmf.NMF_EINVAL),
    ("tol", -1.0, nmf.NMF_EINVAL),
    ("tol", float("inf"), nmf.NMF_EINVAL),
    ("precision", 7, nmf.NMF_EUNSUPPORTED),
    ("tol_kind", 5, nmf.NMF_EUNSUPPORTED),
    ("loss", 3, nmf.NMF_EUNSUPPORTED),
])
def test_init_rejects_bad_options(field, value, code):
    o = nmf.options()
    setattr(o, field, value)
    st, _ = _init(opt=o)
    assert st == code


def test_null_context_calls():
    lib = nmf.load()
    f = ctypes.c_double()
    it = ctypes.c_int32()
    assert lib.nmf_step(None, 1) == nmf.NMF_EINVAL
    assert lib.nmf_update_w(None) == nmf.NMF_EINVAL
    assert lib.nmf_update_h(None) == nmf.NMF_EINVAL
    assert lib.nmf_objective(None, ctypes.byref(f)) == nmf.NMF_EINVAL
    assert lib.nmf_solve(None, 1, ctypes.byref(it), ctypes.byref(f), None, 0) == nmf.NMF_EINVAL
    lib.nmf_destroy(None)  # must not crash


def test_problem_struct_layout_matches_header():
    # three pointers, three int64, two int32 -> 56 bytes
    assert ctypes.sizeof(nmf.NmfProblem) == 56
    assert nmf.NmfProblem.p.offset == 24
    assert nmf.NmfProblem.r.offset == 48


def _batch_create(count=2, out=True, **kw):
    lib = nmf.load()
    arr = (nmf.NmfProblem * max(count, 1))()
    for i in range(max(count, 1)):
        f = dict(V=FAKE, W=FAKE, H=FAKE, p=8, n=8, ldv=8, r=2, reserved=0)
        if i == count - 1:
            f.update(kw)
        arr[i] = nmf.NmfProblem(f["V"], f["W"], f["H"], f["p"], f["n"], f["ldv"], f["r"],
                                f["reserved"])
    b = ctypes.c_void_p(123)
    st = lib.nmf_batch_create(ctypes.byref(b) if out else None, arr, count, None)
    return st, b


@pytest.mark.parametrize("kw", [
    dict(V=None), dict(W=None), dict(H=None), dict(p=0), dict(n=0), dict(r=0), dict(ldv=7),
    dict(V=FAKE + 2), dict(W=FAKE + 1), dict(reserved=1), dict(count=0), dict(count=-1),
    dict(count=16384),
])
def test_batch_create_rejects_bad_arguments(kw):
    st, b = _batch_create(**kw)
    assert st == nmf.NMF_EINVAL
    assert b.value is None


def test_batch_create_rejects_rank_above_64_and_null_out():
    st, _ = _batch_create(r=65)
    assert st == nmf.NMF_EUNSUPPORTED
    st, _ = _batch_create(out=False)
    assert st == nmf.NMF_EINVAL


def test_batch_null_calls():
    lib = nmf.load()
    f = ctypes.c_double()
    t = (ctypes.c_int32 * nmf.BATCH_TABLE_LEN)()
    assert lib.nmf_batch_step(None, 1) == nmf.NMF_EINVAL
    assert lib.nmf_batch_load(None) == nmf.NMF_EINVAL
    assert lib.nmf_batch_check(None) == nmf.NMF_EINVAL
    assert lib.nmf_batch_objective(None, ctypes.byref(f)) == nmf.NMF_EINVAL
    assert lib.nmf_batch_get_table(None, t) == nmf.NMF_EINVAL
    assert lib.nmf_batch_set_table(None, t) == nmf.NMF_EINVAL
    assert lib.nmf_batch_tune(None, 1, None) == nmf.NMF_EINVAL
    assert lib.nmf_batch_solve(None, 1, 1, None, None, None, None) == nmf.NMF_EINVAL
    lib.nmf_batch_destroy(None)  # must not crash


def test_batch_solve_checks_options_before_device_work():
    lib = nmf.load()
    arr = (nmf.NmfProblem * 1)(nmf.NmfProblem(FAKE, FAKE, FAKE, 8, 8, 8, 4, 0))
    for kw, want in ((dict(precision="bf16"), nmf.NMF_EUNSUPPORTED),
                     (dict(check_every=0), nmf.NMF_EINVAL), (dict(tol=-1.0), nmf.NMF_EINVAL)):
        o = nmf.options(**kw)
        assert lib.nmf_batch_solve(arr, 1, 5, ctypes.byref(o), None, None, None) == want, kw
    o = nmf.options(loss="poisson")
    assert lib.nmf_batch_solve(arr, 1, 5, ctypes.byref(o), None, None, None) == \
        nmf.NMF_EUNSUPPORTED
    assert lib.nmf_batch_solve(arr, 1, -1, None, None, None, None) == nmf.NMF_EINVAL
    bad = (nmf.NmfProblem * 1)(nmf.NmfProblem(FAKE, FAKE, FAKE, 8, 8, 8, 65, 0))
    assert lib.nmf_batch_solve(bad, 1, 5, None, None, None, None) == nmf.NMF_EUNSUPPORTED


def test_warm_start_calls_reject_bad_arguments():
    lib = nmf.load()
    P = ctypes.c_void_p
    arr = (P * 1)(FAKE)
    assert lib.nmf_ws_set_dictionary(None, FAKE) == nmf.NMF_EINVAL
    assert lib.nmf_ws_predict(None, FAKE, 8, 8, 8, FAKE, FAKE) == nmf.NMF_EINVAL
    assert lib.nmf_ws_train(None, arr, arr, 1, 8, 8, 8, 1, 8, 1e-3, 1.0, 0, None) == nmf.NMF_EINVAL
    assert lib.nmf_normalize_gauge_noalloc(None, 8, 4, FAKE, 8, None) == nmf.NMF_EINVAL
    assert lib.nmf_normalize_gauge_noalloc(FAKE, 8, 257, FAKE, 8, None) == nmf.NMF_EINVAL
    assert lib.nmf_prepare_graphs(None) == nmf.NMF_EINVAL


@pytest.mark.parametrize("kw", [dict(precision="bf16"), dict(tol_kind="gap"), dict(r=65)])
def test_poisson_loss_rejects_options_it_does_not_offer(kw):
    r = kw.pop("r", 8)
    o = nmf.options(loss="poisson", **kw)
    st, _ = _init(opt=o, r=r)
    assert st == nmf.NMF_EUNSUPPORTED


def test_pet_calls_reject_bad_arguments_before_device_work():
    lib = nmf.load()
    out = ctypes.c_void_p()
    P = ctypes.byref(out)
    # (E, d, p, y, rows, cols, mu, lambda): rows * cols must be p, mu >= 0,
    # pointers non-null and 16-byte aligned, p a multiple of 4
    ok = (FAKE, 10, 12, FAKE, 3, 4, 0.1, FAKE)
    cases = [((None,) + ok[1:], nmf.NMF_EINVAL), (ok[:1] + (0,) + ok[2:], nmf.NMF_EINVAL),
             (ok[:4] + (4, 4) + ok[6:], nmf.NMF_EINVAL), (ok[:6] + (-1.0, FAKE), nmf.NMF_EINVAL),
             (ok[:6] + (float("nan"), FAKE), nmf.NMF_EINVAL),
             (ok[:7] + (FAKE + 4,), nmf.NMF_EINVAL),
             ((FAKE, 10, 10, FAKE, 2, 5, 0.1, FAKE), nmf.NMF_EUNSUPPORTED)]
    for args, code in cases:
        assert lib.nmf_pet_create(P, *args, 0, None) == code, args
        assert not out.value
    assert lib.nmf_pet_create(None, *ok, 0, None) == nmf.NMF_EINVAL
    assert lib.nmf_pet_create(P, *ok, 3, None) == nmf.NMF_EINVAL      # unknown layout
    assert lib.nmf_pet_layout(None, ctypes.byref(ctypes.c_int32())) == nmf.NMF_EINVAL
    f, it = ctypes.c_double(), ctypes.c_int32()
    assert lib.nmf_pet_step(None, 1) == nmf.NMF_EINVAL
    assert lib.nmf_pet_objective(None, ctypes.byref(f)) == nmf.NMF_EINVAL
    assert lib.nmf_pet_solve(None, 10, 1e-9, 1, ctypes.byref(it), ctypes.byref(f)) == \
        nmf.NMF_EINVAL
    lib.nmf_pet_destroy(None)


def test_ceiling_rejects_bad_arguments_before_device_work():
    lib = nmf.load()
    rate = ctypes.c_double(-1.0)
    R = ctypes.byref(rate)
    big = 64 << 20
    cases = [(-1, FAKE, big, 5, R), (7, FAKE, big, 5, R),          # unknown kind
             (0, None, big, 5, R), (1, FAKE, big, 5, None),        # null pointers
             (1, FAKE, big - 256, 5, R), (1, FAKE, big + 8, 5, R),  # too small, not 256-aligned
             (2, FAKE, big, 0, R), (2, FAKE, big, 1001, R),        # reps out of range
             (3, FAKE + 16, big, 5, R)]                           # buffer not 256-aligned
    for args in cases:
        assert lib.nmf_ceiling(*args, None) == nmf.NMF_EINVAL, args
    assert rate.value == -1.0
