"""The allocation-free energy entry point (tmop_energy_noalloc) against
tmop_energy through the C ABI: the same kernels and reduction order, so F
and min det A agree bit for bit; two calls in a row on meshes of different
sizes (the second smaller, then the larger again), objectives with several
terms, and the size limit."""
import ctypes

import numpy as np
import pytest

from paper_1807_09807_amd import meshgen
from tests._helpers import say, to_dev

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _ctx(dim, n, p, Q, metric, seed, precision=0):
    from paper_1807_09807_amd import tmop as T
    mesh = meshgen.box_mesh(dim, n, p)
    x = meshgen.perturb(mesh, 0.05, seed)
    ctx = T.Context(dim, p, mesh.elem_node, mesh.n_node, Q, metric, mesh.h * np.eye(dim), fixed=mesh.fixed,
                    precision=precision)
    return mesh, ctx, to_dev(x)


def _call_noalloc(ctx, x):
    """Straight through the C ABI."""
    from paper_1807_09807_amd import tmop as T
    lib = T.load()
    F, md = ctypes.c_double(), ctypes.c_double()
    st = lib.tmop_energy_noalloc(ctx.handle, ctypes.c_void_p(x.data_ptr()), ctypes.byref(F), ctypes.byref(md),
                                 ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    return st, F.value, md.value


def _check(ctx, x, label):
    st, F, md = _call_noalloc(ctx, x)
    Fr, mdr, str_ = ctx.energy(x)
    say(f"  {label}: noalloc F {F!r} min det {md!r} status {st}; energy F {Fr!r} status {str_}")
    assert st == str_ == 0
    assert F == Fr and md == mdr


def test_noalloc_matches_energy_two_calls():
    say("[noalloc] 3D 16^3 Q2, then 2D 8^2 Q2, then 3D again")
    big = _ctx(3, 16, 2, 4, 303, 1)
    small = _ctx(2, 8, 2, 4, 2, 2)
    _check(big[1], big[2], "3D 16^3 Q2 (1024 workgroups)")
    _check(small[1], small[2], "2D 8^2 Q2")
    _check(big[1], big[2], "3D 16^3 Q2 again")
    big[1].close()
    small[1].close()


@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "mixed"])
def test_noalloc_with_section4_terms(precision):
    """Three terms (primary, eq. 4.1 second term, eq. 4.2 penalty): their
    partials sit side by side in the scratch."""
    say(f"[noalloc] 2D 12^2 Q3 mu_7 + mu_2 + penalty, precision {precision}")
    mesh, ctx, x = _ctx(2, 12, 3, 5, 7, 3, precision)
    ctx.set_combo(2, mesh.h * np.array([[1.0, 0.3], [0.0, 1.2]]), eta1=1.0, eta2=0.5)
    ctx.set_restriction(3.0, to_dev(mesh.x_grid))
    _check(ctx, x, "three terms")
    small = _ctx(3, 3, 2, 4, 302, 4, precision)
    _check(small[1], small[2], "3D 3^3 Q2 after it")
    small[1].close()
    ctx.close()


def test_noalloc_size_limit():
    """64^3 Q2 hexahedra with 4^3 points need exactly the 65,536 workgroups
    the scratch holds; 65^3 need more and are refused before any device work."""
    from paper_1807_09807_amd import tmop as T
    say("[noalloc] 64^3 Q2 (at the limit) and 65^3 Q2 (over it)")
    for n, expect in ((64, T.TMOP_OK), (65, T.TMOP_E_SCRATCH)):
        mesh = meshgen.box_mesh(3, n, 2)
        ctx = T.Context(3, 2, mesh.elem_node, mesh.n_node, 4, 303, mesh.h * np.eye(3))
        x = to_dev(mesh.x_grid)
        st, F, md = _call_noalloc(ctx, x)
        say(f"  {n}^3: status {st}")
        assert st == expect
        if expect == T.TMOP_OK:
            Fr, mdr, _ = ctx.energy(x)
            assert F == Fr and md == mdr
        with pytest.raises(T.TMOPError) if expect != T.TMOP_OK else _noop():
            ctx.energy_noalloc(x)
        ctx.close()
        del x
        torch.cuda.empty_cache()


class _noop:
    def __enter__(self):
        return self

    def __exit__(self, *a):
        return False
