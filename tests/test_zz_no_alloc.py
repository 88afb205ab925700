"""hpf_relax_async_noalloc (the entry point for callers that cannot
allocate): through the C ABI, its results equal hpf_relax_async's bit for bit
on two calls in a row (the second on a smaller grid), it can be captured into
a graph at the first call of a grid size, and it rejects grids beyond its
static scratch."""
import numpy as np
import pytest
import torch

from paper_1903_07441_amd import scenarios
from test_gpu_relax import to_dev

pytestmark = pytest.mark.gpu

KEYS = ("sweeps", "polish_sweeps", "residual", "residual32", "cert_bound", "status", "polish_rounds", "checks",
        "omega")


def _case(orc, name, idx, side=None, pitch=None):
    sc = scenarios.scenario(name, idx, side=side)
    cls, _ = orc.rasterize(sc)
    ny, nx = cls.shape
    pitch = pitch or nx
    c = to_dev(cls, pitch)
    return cls, c, ny, nx, pitch


def _fields(ny, pitch):
    return (torch.zeros((ny, pitch), dtype=torch.float32, device="cuda"),
            torch.zeros((ny, pitch), dtype=torch.float64, device="cuda"))


def _views(psi, psi64, nx):
    return psi[:, :nx], psi64[:, :nx]


@pytest.mark.parametrize("polish", [0, 1])
def test_noalloc_equals_async_two_calls(ctx, orc, polish):
    from paper_1903_07441_amd import twg
    kw = dict(tol=1e-6, polish=polish, tol_cert=5e-7 if polish else 0.0)
    # a 512 x 512 grid, then a smaller, ragged one (odd width, padded pitch)
    for name, idx, side, pitch in (("warped512", 0, None, None), ("warped512", 3, 301, 320)):
        cls, c, ny, nx, pitch = _case(orc, name, idx, side, pitch)
        print(f"noalloc vs async: {name}[{idx}] {nx}x{ny} pitch {pitch} polish {polish}", flush=True)
        pa, pa64 = _fields(ny, pitch)
        va, va64 = _views(pa, pa64, nx)
        sa = twg.stats_from_device(ctx.relax_async(c[:, :nx], va, va64 if polish else None, slots=4000, **kw))
        pn, pn64 = _fields(ny, pitch)
        vn, vn64 = _views(pn, pn64, nx)
        stats = torch.zeros(twg.STATS_BYTES, dtype=torch.uint8, device="cuda")
        ctx.relax_async(c[:, :nx], vn, vn64 if polish else None, slots=4000, stats=stats, noalloc=True, **kw)
        sn = twg.stats_from_device(stats)
        print(f"  async {sa}\n  noalloc {sn}", flush=True)
        assert sa["status"] == twg.OK
        for k in KEYS:
            assert sn[k] == sa[k], k
        assert torch.equal(pn, pa)
        if polish:
            assert torch.equal(pn64, pa64)
            # the certificate, recomputed by the oracle
            r = orc.residual(cls, vn64.cpu().numpy())
            assert r * orc.wbound(nx, ny) <= 5e-7
        else:
            assert orc.residual(cls, vn.cpu().numpy().astype(np.float64)) <= 1e-6


def test_noalloc_captured_at_first_call_of_a_size(ctx, orc):
    """Captured into a graph at a grid size no call of this process has used
    (nothing can be allocated then), the replays give the bits of an eager
    hpf_relax_async call, with eager work and synchronisations between
    replays."""
    from paper_1903_07441_amd import twg
    cls, c, ny, nx, pitch = _case(orc, "warped512", 5, 200)
    kw = dict(tol=1e-6, polish=1, tol_cert=5e-7)
    psi, psi64 = _fields(ny, pitch)
    stats = torch.zeros(twg.STATS_BYTES, dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        ctx.relax_async(c, psi, psi64, slots=1500, stats=stats, noalloc=True, **kw)
    pe, pe64 = _fields(ny, pitch)
    se = twg.stats_from_device(ctx.relax_async(c, pe, pe64, slots=1500, **kw))
    assert se["status"] == twg.OK
    for rep in range(3):
        psi.fill_(-3.0)
        psi64.fill_(-3.0)
        stats.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        sr = twg.stats_from_device(stats)
        print(f"replay {rep}: {sr}", flush=True)
        for k in KEYS:
            assert sr[k] == se[k], (rep, k)
        assert torch.equal(psi, pe) and torch.equal(psi64, pe64)
        # eager work between replays, on the same static scratch
        junk, _ = _fields(ny, pitch)
        st2 = torch.zeros(twg.STATS_BYTES, dtype=torch.uint8, device="cuda")
        ctx.relax_async(c, junk, None, slots=200, stats=st2, tol=1e-4, noalloc=True)
        torch.cuda.synchronize()
    del g


def test_noalloc_rejects_grids_beyond_its_scratch(ctx):
    from paper_1903_07441_amd import twg
    ny, nx = 2048, 2049  # pitch * ny = 4196352 > 2^22
    c = torch.zeros((ny, nx), dtype=torch.uint8, device="cuda")
    psi = torch.zeros((ny, nx), dtype=torch.float32, device="cuda")
    stats = torch.zeros(twg.STATS_BYTES, dtype=torch.uint8, device="cuda")
    with pytest.raises(twg.TwgError) as e:
        ctx.relax_async(c, psi, None, slots=10, stats=stats, noalloc=True)
    assert e.value.code == twg.EUNSUPPORTED
    assert "4194304" in str(e.value)
