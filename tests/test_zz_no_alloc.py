"""p3t_long_force_vjp_noalloc through the C ABI: the same VJP as
p3t_long_force_vjp (same kernels, workspaces in the library's static
per-device array), with no call of the context allocator.

Two calls in a row on one context, the second on a smaller build, so that a
value left in the shared workspace by the first call would show in the second;
each against p3t_long_force_vjp on the same build.  Also: a build too large
for the static workspace is rejected (ECAPACITY, outputs untouched), and so is
a call after the lists were released (ESTATE).
"""
import ctypes as C

import numpy as np
import pytest

from inputs import plummer
from tests.gpu_cases import log

pytestmark = pytest.mark.gpu

P3T_ESTATE, P3T_ECAPACITY = -4, -3


class CountingContext:
    """A raw library context whose allocator counts its calls."""

    def __init__(self):
        import torch
        from paper_1506_04553_amd import load_library
        from paper_1506_04553_amd.p3t import ALLOC_FN, FREE_FN
        self.L = load_library()
        self.allocs = 0
        self.frees = 0
        stream = torch.cuda.current_stream(0)

        def _alloc(nbytes, _user):
            self.allocs += 1
            return torch.cuda.caching_allocator_alloc(int(nbytes), 0, stream)

        def _free(p, _user):
            self.frees += 1
            torch.cuda.caching_allocator_delete(int(p))

        self._cb = (ALLOC_FN(_alloc), FREE_FN(_free))
        h = C.c_void_p()
        assert self.L.p3t_create(C.byref(h), 0, C.c_void_p(stream.cuda_stream), *self._cb, None) == 0
        self.h = h

    def check(self, rc):
        if rc != 0:
            raise AssertionError(f"status {rc}: {self.L.p3t_last_error(self.h).decode()}")

    def close(self):
        self.L.p3t_destroy(self.h)


def _p(ptr_of):
    return C.c_void_p(ptr_of.data_ptr()) if ptr_of is not None else None


def _build(cx, pos, mass, precision, r_out=0.01):
    from paper_1506_04553_amd import make_params
    n = len(mass)
    prm = make_params(eps=4.0 / n, r_in=0.1 * r_out, r_out=r_out, theta=0.5, r_search=1.1 * r_out,
                      n_crit=64, n_leaf=16, precision=precision)
    cx.check(cx.L.p3t_build_tree(cx.h, n, _p(pos), _p(mass), C.byref(prm)))


def _close(a, b, label):
    """The two calls differ only in the order of the FP64 atomic additions of
    the scatter pass (1e-16 of each term, where the terms of one coordinate
    cancel by up to three orders of magnitude): relative RMS 1e-12, and element
    by element, relative to the larger of the element and 1e-3 of the RMS,
    the FP64 VJP's per-row bound of 1e-9."""
    scale = np.sqrt(np.mean(b ** 2))
    err = np.abs(a - b) / (np.abs(b) + 1e-3 * scale)
    rms = np.sqrt(np.mean((a - b) ** 2)) / scale
    log(f"  {label}: rel-RMS {rms:.2e}, max element error {err.max():.2e}")
    assert np.all(np.isfinite(a)), label
    assert rms < 1e-12 and err.max() < 1e-9, label


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_noalloc_vjp_matches_vjp(precision):
    import torch
    dev = torch.device("cuda", 0)
    cx = CountingContext()
    try:
        for n, seed, with_c in ((40000, 11, True), (6000, 12, False)):
            log(f"noalloc vjp {precision} n={n} c={'yes' if with_c else 'no'}")
            cl = plummer(n, seed)
            pos = torch.from_numpy(cl.pos).to(dev)
            mass = torch.from_numpy(cl.mass).to(dev)
            rng = np.random.default_rng(seed + 100)
            w = torch.from_numpy(rng.normal(size=(n, 3))).to(dev)
            cw = torch.from_numpy(rng.normal(size=n)).to(dev) if with_c else None
            _build(cx, pos, mass, precision)
            gp_ref = torch.empty((n, 3), dtype=torch.float64, device=dev)
            gm_ref = torch.empty((n,), dtype=torch.float64, device=dev)
            cx.check(cx.L.p3t_long_force_vjp(cx.h, _p(w), _p(cw), _p(gp_ref), _p(gm_ref)))
            gp = torch.full((n, 3), float("nan"), dtype=torch.float64, device=dev)
            gm = torch.full((n,), float("nan"), dtype=torch.float64, device=dev)
            torch.cuda.synchronize()
            allocs, frees = cx.allocs, cx.frees
            cx.check(cx.L.p3t_long_force_vjp_noalloc(cx.h, _p(w), _p(cw), _p(gp), _p(gm)))
            torch.cuda.synchronize()
            assert (cx.allocs, cx.frees) == (allocs, frees), "the no-allocation call allocated"
            _close(gp.cpu().numpy(), gp_ref.cpu().numpy(), "gpos")
            _close(gm.cpu().numpy(), gm_ref.cpu().numpy(), "gmass")
    finally:
        cx.close()


def test_noalloc_vjp_rejects_what_it_cannot_hold():
    import torch
    dev = torch.device("cuda", 0)
    cx = CountingContext()
    try:
        # 4 n + 10 n_nodes doubles above the 64 MiB workspace: ECAPACITY
        n = 1 << 21
        log(f"noalloc vjp capacity n={n}")
        rng = np.random.default_rng(5)
        pos = torch.from_numpy(rng.uniform(-1.0, 1.0, (n, 3))).to(dev)
        mass = torch.full((n,), 1.0 / n, dtype=torch.float64, device=dev)
        _build(cx, pos, mass, "mixed", r_out=0.002)
        w = torch.ones((n, 3), dtype=torch.float64, device=dev)
        gp = torch.full((n, 3), 7.0, dtype=torch.float64, device=dev)
        gm = torch.full((n,), 7.0, dtype=torch.float64, device=dev)
        rc = cx.L.p3t_long_force_vjp_noalloc(cx.h, _p(w), None, _p(gp), _p(gm))
        assert rc == P3T_ECAPACITY, rc
        assert b"static workspace" in cx.L.p3t_last_error(cx.h)
        torch.cuda.synchronize()
        assert bool((gp == 7.0).all()) and bool((gm == 7.0).all())
        del pos, mass, w, gp, gm
        # released lists: walking again would allocate, so ESTATE
        n = 3000
        cl = plummer(n, 13)
        pos = torch.from_numpy(cl.pos).to(dev)
        mass = torch.from_numpy(cl.mass).to(dev)
        _build(cx, pos, mass, "fp64")
        cx.check(cx.L.p3t_release_lists(cx.h))
        w = torch.from_numpy(np.random.default_rng(6).normal(size=(n, 3))).to(dev)
        gp = torch.empty((n, 3), dtype=torch.float64, device=dev)
        gm = torch.empty((n,), dtype=torch.float64, device=dev)
        assert cx.L.p3t_long_force_vjp_noalloc(cx.h, _p(w), None, _p(gp), _p(gm)) == P3T_ESTATE
        # the ordinary call walks again; after it the lists are back
        cx.check(cx.L.p3t_long_force_vjp(cx.h, _p(w), None, _p(gp), _p(gm)))
        gp2 = torch.empty_like(gp)
        gm2 = torch.empty_like(gm)
        cx.check(cx.L.p3t_long_force_vjp_noalloc(cx.h, _p(w), None, _p(gp2), _p(gm2)))
        torch.cuda.synchronize()
        _close(gp2.cpu().numpy(), gp.cpu().numpy(), "gpos after release")
    finally:
        cx.close()
