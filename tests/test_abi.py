"""The C ABI without a GPU: the library loads, exports every declared symbol,
and rejects invalid arguments before any HIP call."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lagp_alc.h")


@pytest.fixture(scope="module")
def L():
    from paper_1310_5182_amd import _lib

    return _lib.load()


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lagp_\w+)\s*\(", text)))


def test_header_declares_entry_points():
    syms = declared_symbols()
    for s in ("lagp_nn_pool", "lagp_alc_from_pool", "lagp_alc_predict", "lagp_last_error"):
        assert s in syms


def test_exports_every_declared_symbol(L):
    from paper_1310_5182_amd import _lib

    for s in declared_symbols():
        assert hasattr(L, s), s
    assert sorted(_lib.EXPORTS) == declared_symbols()


def test_version_and_strings(L):
    assert b"gfx950" in L.lagp_version()
    assert L.lagp_status_string(0) == b"LAGP_OK"
    assert L.lagp_status_string(-1) == b"LAGP_EINVAL"
    assert L.lagp_status_string(-4) == b"LAGP_EUNSUPPORTED"


FAKE = 0x1000  # never dereferenced: validation fails (or M == 0) before any HIP call


def nn(L, N=100, p=2, M=3, Np=10, X=FAKE, XX=FAKE, pool=FAKE):
    return L.lagp_nn_pool(X, N, p, XX, M, Np, pool, None)


def alc(L, N=100, p=2, M=3, Np=10, n0=2, n=5, d=0.5, g=1e-3, prec=0, Y=FAKE, sel=FAKE):
    return L.lagp_alc_from_pool(FAKE, Y, N, p, FAKE, M, FAKE, Np, n0, n, d, g, prec,
                                None, None, None, sel, None, None, None, None, None)


def test_nn_pool_validation(L):
    assert nn(L, Np=0) == -1
    assert nn(L, Np=101) == -1
    assert nn(L, p=0) == -1
    assert nn(L, N=0) == -1
    assert nn(L, M=-1) == -1
    assert nn(L, pool=None) == -1
    assert nn(L, X=None) == -1
    assert nn(L, p=17) == -4
    assert nn(L, N=10**6, Np=5000) == -4
    assert b"Np" in L.lagp_last_error()
    assert nn(L, M=0) == 0  # no-op, no HIP call
    assert L.lagp_last_error() == b""


def test_alc_validation(L):
    assert alc(L, n0=0) == -1
    assert alc(L, n0=6, n=5) == -1
    assert alc(L, n=11) == -1
    assert alc(L, d=0.0) == -1
    assert alc(L, d=float("nan")) == -1
    assert alc(L, g=0.0) == -1
    assert alc(L, g=float("inf")) == -1
    assert alc(L, prec=3) == -1
    assert alc(L, Y=None) == -1
    assert alc(L, sel=None) == -1
    assert alc(L, N=5000, Np=2000, n=50) == -4
    assert alc(L, N=5000, n=130, Np=200, prec=0) == -4
    assert alc(L, p=9) == -4
    assert alc(L, M=0) == 0


def problem(**kw):
    from paper_1310_5182_amd import _lib

    pr = _lib.Problem()
    pr.struct_size = ctypes.sizeof(_lib.Problem)
    vals = dict(X=FAKE, Y=FAKE, XX=FAKE, N=100, M=3, p=2, n0=6, n=20, Np=50, d=0.5, g=1e-3, precision=0, flags=0)
    vals.update(kw)
    for k, v in vals.items():
        setattr(pr, k, v)
    return pr


def outputs(**kw):
    from paper_1310_5182_amd import _lib

    po = _lib.Outputs()
    po.struct_size = ctypes.sizeof(_lib.Outputs)
    po.sel = FAKE
    for k, v in kw.items():
        setattr(po, k, v)
    return po


def predict(L, pr, po, ws=FAKE * 256, nbytes=1 << 40):
    return L.lagp_alc_predict(ctypes.byref(pr) if pr is not None else None,
                              ctypes.byref(po) if po is not None else None, ws, nbytes, None)


def test_struct_layout_and_abi_guard(L):
    from paper_1310_5182_amd import _lib

    # the ctypes mirrors have the C layout (the library accepts exactly these sizes)
    assert ctypes.sizeof(_lib.Problem) == 120 and ctypes.sizeof(_lib.Outputs) == 88
    assert L.lagp_abi_version() == _lib.LAGP_ABI_VERSION == 3
    assert predict(L, problem(M=0), outputs()) == 0
    assert L.lagp_last_error() == b""
    for bad in (0, 112, 128):  # 112: the version-2 layout, without d_sep
        assert predict(L, problem(M=0, struct_size=bad), outputs()) == -1
        assert b"struct_size" in L.lagp_last_error()
    for bad in (0, 80, 96):
        assert predict(L, problem(M=0), outputs(struct_size=bad)) == -1
        assert b"lagp_outputs.struct_size" in L.lagp_last_error()
    nb = ctypes.c_size_t(0)
    assert L.lagp_alc_workspace(ctypes.byref(problem(struct_size=8)), ctypes.byref(nb)) == -1


def test_separable_validation(L):
    """d_sep (the separable kernel) needs LAGP_FP64 and excludes d_per."""
    assert predict(L, problem(d_sep=FAKE, precision=1), outputs()) == -4
    assert b"d_sep" in L.lagp_last_error()
    assert predict(L, problem(d_sep=FAKE, precision=2), outputs()) == -4
    assert predict(L, problem(d_sep=FAKE, d_per=FAKE), outputs()) == -1
    assert predict(L, problem(d_sep=FAKE, M=0), outputs()) == 0


def test_predict_validation(L):
    assert predict(L, None, outputs()) == -1
    assert predict(L, problem(), None) == -1
    assert predict(L, problem(), outputs(sel=None)) == -1
    assert predict(L, problem(flags=8), outputs()) == -1            # unknown flag
    assert predict(L, problem(reserved=1), outputs()) == -1
    assert predict(L, problem(), outputs(reserved=1)) == -1
    assert predict(L, problem(n0=0), outputs()) == -1
    assert predict(L, problem(n=51), outputs()) == -1               # n above N'
    assert predict(L, problem(Np=101), outputs()) == -1             # N' above N
    assert predict(L, problem(d=0.0), outputs()) == -1
    assert predict(L, problem(g=float("nan")), outputs()) == -1
    assert predict(L, problem(precision=3), outputs()) == -1
    assert predict(L, problem(p=9), outputs()) == -4
    assert predict(L, problem(Y=None), outputs()) == -1
    # the normalisation of Fig. 3 step 9 divides by j - 2
    assert predict(L, problem(flags=1, n0=2), outputs()) == -1
    assert b"n0 >= 3" in L.lagp_last_error()
    assert predict(L, problem(flags=1, n0=3, M=0), outputs()) == 0
    # the re-forming kernels take uniform sizes only
    assert predict(L, problem(precision=2, n_per=FAKE), outputs()) == -4
    assert predict(L, problem(precision=2), outputs(sel_off=FAKE)) == -4
    assert predict(L, problem(N=10**5, n=129, Np=2000), outputs()) == -4
    assert predict(L, problem(N=10**5, Np=4096), outputs()) == -4
    assert predict(L, problem(M=0, precision=1), outputs()) == 0


def test_predict_workspace(L):
    nb = ctypes.c_size_t(0)
    assert L.lagp_alc_workspace(None, ctypes.byref(nb)) == -1
    assert L.lagp_alc_workspace(ctypes.byref(problem()), None) == -1
    # uniform float64 sizes: no queue, so the query needs no device
    assert L.lagp_alc_workspace(ctypes.byref(problem(flags=2)), ctypes.byref(nb)) == 0
    assert nb.value == 768                                        # the pools, 3 x 50 int32, 256-aligned
    assert L.lagp_alc_workspace(ctypes.byref(problem()), ctypes.byref(nb)) == 0
    grid = ctypes.c_size_t(0)
    assert L.lagp_nn_pool_workspace(100, 2, 3, ctypes.byref(grid)) == 0
    assert nb.value >= grid.value + 3 * 50 * 4
    need = nb.value
    assert predict(L, problem(), outputs(), nbytes=need - 1) == -2
    assert predict(L, problem(), outputs(), ws=FAKE * 256 + 16, nbytes=need) == -2   # not 256-byte aligned
    assert predict(L, problem(), outputs(), ws=None, nbytes=need) == -2
    assert b"256-byte aligned" in L.lagp_last_error()


def test_python_binding_rejects_cpu_tensors():
    import torch

    import paper_1310_5182_amd as lagp

    with pytest.raises(ValueError):
        lagp.nn_pool(torch.zeros(10, 2, dtype=torch.float64), torch.zeros(2, 2, dtype=torch.float64), 3)


def test_local_validation(L):
    P = FAKE
    # n outside [1, 64]
    assert L.lagp_local_nll(P, P, 100, 2, P, 3, 0, P, P, P, None, None, None, None, None) == -1
    assert L.lagp_local_nll(P, P, 100, 2, P, 3, 65, P, P, P, None, None, None, None, None) == -4
    assert L.lagp_local_nll(P, P, 100, 2, None, 3, 10, P, P, P, None, None, None, None, None) == -1
    assert L.lagp_local_nll(P, P, 100, 2, P, 0, 10, P, P, P, None, None, None, None, None) == 0
    # MLE bounds and nugget
    assert L.lagp_local_mle_d(P, P, 100, 2, P, 3, 10, P, 1e-3, 0.0, 5.0, 100, P, None, None, None, None) == -1
    assert L.lagp_local_mle_d(P, P, 100, 2, P, 3, 10, P, 1e-3, 1.0, 0.5, 100, P, None, None, None, None) == -1
    assert L.lagp_local_mle_d(P, P, 100, 2, P, 3, 10, P, 0.0, 1e-3, 5.0, 100, P, None, None, None, None) == -1
    assert L.lagp_local_mle_d(P, P, 100, 2, P, 3, 10, P, 1e-3, 1e-3, 5.0, -1, P, None, None, None, None) == -1
    assert L.lagp_local_predict(P, P, 100, 2, P, 3, 10, None, P, 1e-3, None, None, None, None, None) == -1
    assert L.lagp_local_nll_backward(P, P, 100, 2, P, 3, 10, None, P, None, P, P, None) == -1


def uneven(L, N=5000, p=4, M=3, Np=2000, n0=6, n=100, prec=0, ws=FAKE, nbytes=1 << 30, sel=FAKE):
    return L.lagp_alc_uneven_from_pool(FAKE, FAKE, N, p, FAKE, M, FAKE, Np, n0, n, None, None, None, None,
                                       0.3, 1e-5, prec, None, None, None, sel, None, None, None,
                                       ws, nbytes, None)


def test_uneven_validation(L):
    nb = ctypes.c_size_t(0)
    assert L.lagp_alc_uneven_workspace(4, 10, 2000, 100, None) == -1
    assert L.lagp_alc_uneven_workspace(4, -1, 2000, 100, ctypes.byref(nb)) == -1
    assert L.lagp_alc_uneven_workspace(9, 10, 2000, 100, ctypes.byref(nb)) == -4
    assert L.lagp_alc_uneven_workspace(4, 10, 2049, 100, ctypes.byref(nb)) == -4
    assert L.lagp_alc_uneven_workspace(4, 10, 2000, 129, ctypes.byref(nb)) == -4
    assert uneven(L, prec=1) == -4          # float64 only
    assert uneven(L, prec=3) == -1
    assert uneven(L, n=129) == -4
    assert uneven(L, N=10000, Np=2049) == -4
    assert uneven(L, p=9) == -4
    assert uneven(L, n0=0) == -1
    assert uneven(L, n=2001) == -1          # n_max above the pool width
    assert uneven(L, sel=None) == -1
    assert uneven(L, M=0) == 0


def test_plan_validation(L):
    h = ctypes.c_void_p()

    def create(pr, po=None, handle=True, flags=0):
        po = po or outputs()
        return L.lagp_plan_create(ctypes.byref(pr) if pr is not None else None, ctypes.byref(po), FAKE * 256,
                                  1 << 40, flags, None, ctypes.byref(h) if handle else None)

    assert create(problem(), handle=False) == -1                     # no handle
    assert create(None) == -1
    assert create(problem(M=0)) == -1                                 # a plan needs M >= 1
    assert b"M >= 1" in L.lagp_last_error()
    assert create(problem(N=5000, n=129, Np=2000)) == -4              # n beyond 128
    assert create(problem(n0=0)) == -1
    assert create(problem(struct_size=96)) == -1
    assert create(problem(), flags=4) == -1                           # unknown plan flag
    assert create(problem(), flags=7 << 8) == -1                      # LAGP_PLAN_SCHEDULE(6): no such schedule
    assert b"LAGP_PLAN_SCHEDULE" in L.lagp_last_error()
    assert h.value is None
    assert L.lagp_plan_destroy(None) == 0
    assert L.lagp_plan_launch(None, None) == -1


def test_nn_pool_ws_validation(L):
    nb = ctypes.c_size_t(0)
    assert L.lagp_nn_pool_workspace(100, 2, 3, None) == -1
    assert L.lagp_nn_pool_workspace(100, 17, 3, ctypes.byref(nb)) == -4
    assert L.lagp_nn_pool_workspace(0, 2, 3, ctypes.byref(nb)) == -1
    assert L.lagp_nn_pool_workspace(100, 2, -1, ctypes.byref(nb)) == -1
    assert L.lagp_nn_pool_workspace(100, 3, 3, ctypes.byref(nb)) == 0
    need = nb.value
    assert need >= 100 * (3 * 4 + 8)                              # rows cell by cell, indices, cells
    assert L.lagp_nn_pool_workspace(200, 3, 3, ctypes.byref(nb)) == 0 and nb.value > need
    assert L.lagp_nn_pool_workspace(100, 3, 3000, ctypes.byref(nb)) == 0 and nb.value > need
    ws = lambda *a: L.lagp_nn_pool_ws(*a, None)                   # noqa: E731
    assert ws(FAKE, 100, 3, FAKE, 3, 10, FAKE, FAKE, need - 1) == -2  # too small
    assert ws(FAKE, 100, 3, FAKE, 3, 10, FAKE, FAKE + 4, need) == -2  # not 16-byte aligned
    assert ws(FAKE, 100, 3, FAKE, 3, 10, FAKE, None, need) == -2
    assert ws(FAKE, 100, 3, FAKE, 3, 101, FAKE, FAKE, need) == -1
    assert ws(FAKE, 100, 3, FAKE, 3, 10, None, FAKE, need) == -1
    assert ws(FAKE, 10**6, 3, FAKE, 3, 5000, FAKE, FAKE, 1 << 30) == -4
    assert ws(FAKE, 100, 3, FAKE, 0, 10, FAKE, None, 0) == 0     # M = 0: no-op


def test_scores_validation(L):
    P = FAKE
    sc = lambda j=4, p=2, Nc=10, d=0.5, g=1e-3, prec=0, delta=P: L.lagp_alc_scores(  # noqa: E731
        P, j, p, P, P, Nc, P, P, d, g, prec, delta, None)
    assert sc(j=0) == -1
    assert sc(j=513) == -4
    assert b"512" in L.lagp_last_error()
    assert sc(p=0) == -1
    assert sc(p=17) == -4
    assert sc(Nc=-1) == -1
    assert sc(d=0.0) == -1
    assert sc(g=float("nan")) == -1
    assert sc(prec=2) == -1
    assert sc(delta=None) == -1
    assert sc(Nc=0, delta=None) == 0     # no-op before any pointer is needed


def mspe(L, N=100, p=2, M=3, Np=10, n0=2, n=5, d=0.5, g=1e-3, ws=FAKE, ws_bytes=1 << 40):
    return L.lagp_mspe_from_pool(FAKE, FAKE, N, p, FAKE, M, FAKE, Np, n0, n, d, g, None, None, None, FAKE, None,
                                 None, ws, ws_bytes, None)


def test_mspe_validation(L):
    import ctypes as ct

    assert mspe(L, n0=1) == -1  # eq. newv divides by j (j - 1)
    assert b"n0 >= 2" in L.lagp_last_error()
    assert mspe(L, n0=6, n=5) == -1
    assert mspe(L, n=11) == -1
    assert mspe(L, d=0.0) == -1
    assert mspe(L, g=-1.0) == -1
    assert mspe(L, N=10**6, Np=2000, n=10) == -4
    assert mspe(L, N=10**6, Np=500, n=65) == -4
    assert mspe(L, p=9) == -4
    assert mspe(L, M=0) == 0  # no-op, no HIP call
    nb = ct.c_size_t(7)
    assert L.lagp_mspe_workspace(0, 10, 5, ct.byref(nb)) == 0 and nb.value == 0
    assert L.lagp_mspe_workspace(10, 2000, 5, ct.byref(nb)) == -4
    assert L.lagp_mspe_workspace(10, 10, 5, None) == -1


def test_nn_pool_grouped_validation(L):
    def grouped(group, p=2, Np=10, M=3, ws=FAKE, nbytes=1 << 40):
        return L.lagp_nn_pool_grouped(FAKE, 100, p, FAKE, M, Np, group, FAKE, ws, nbytes, None)

    assert grouped(3) == -1
    assert grouped(0) == -1
    assert grouped(2, p=9) == -4                 # grouped pools are compiled for p <= 8
    assert grouped(2, M=0) == 0
    assert grouped(4, M=3, ws=None) == -2
