"""Lattices as large as the device's memory holds, where every offset in the
step kernels passes 32 bits: FP16 at 65536 x 65536 (2^32 nodes, two 77.3 GB
population buffers) and FP32 at 46400 x 46400 (2.15e9 > 2^31 nodes, two
77.5 GB buffers).  Each starts from seeded uniform-noise velocity (|u_x|,
|u_y| <= 0.03; Grad initialisation with central differences; KBC-B,
nu = 1e-4), takes one step with the single-step kernel and then two in one
fused launch (the default configuration), and is checked after each against
the oracle run on a periodic window around sampled nodes: the four corners,
the edges, the rows that hold element offsets 2^31 and 2^32, byte offsets
2^32 and node index 2^31, tile edges, and random nodes.  The populations are
read straight from the storage buffer and decoded as the storage is defined
(f_i(x) is stored at x - v_i, as binary16 g_i 2^s_i or binary32 g_i, with
f_i = g_i + W_i): the FP64 export of the whole lattice would need 309 GB.

Bars as at 16384^2 (max |gpu - oracle| / max |oracle - W| over the samples):
FP32 2e-5 after one step and 1e-4 after three, FP16 5e-3 and 1e-2, or five
times the oracle's own movement when its stored states are rounded to the
form, if that is larger."""
import sys

import numpy as np
import pytest
import torch

from paper_1507_02509_amd import inputs
from paper_1507_02509_amd.sim import Sim, beta_from_nu
from oracle_sensitivity import K_SENS

pytestmark = pytest.mark.gpu

W = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
SHIFT = np.array([1, 3, 3, 3, 3, 5, 5, 5, 5])       # binary16 storage scale exponents
CX = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1])
CY = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1])
TOL1 = {"f32": 2e-5, "f16": 5e-3}
TOL3 = {"f32": 1e-4, "f16": 1e-2}
AMP, NU, SEED = 0.03, 1e-4, 41
STORE_BYTES = {"f16": 2, "f32": 4}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def sample_nodes(nx, ny, pitch, elem_bytes):
    """Corners, edges, tile edges, the rows holding the 32-bit crossings of
    element offsets, byte offsets and node indices (and the rows next to
    them), and random nodes."""
    row_elems = 9 * pitch                   # elements of one lattice row [9][pitch]
    rows = {0, 1, 15, 16, ny // 2, ny - 2, ny - 1}
    for e in (1 << 31, 1 << 32):            # element offsets
        rows |= {e // row_elems, e // row_elems + 1}
    rows.add((1 << 32) // elem_bytes // row_elems)   # byte offset 2^32
    if nx * ny > (1 << 31):
        rows |= {(1 << 31) // nx, (1 << 31) // nx + 1}   # node index 2^31
    rows = sorted(r for r in rows if 0 <= r < ny)
    cols = [0, 63, 64, nx // 2, nx - 1]
    pts = [(x, y) for y in rows for x in (cols if y in (0, ny - 1) else (0, nx - 1, 64 + y % 500))]
    rng = np.random.default_rng(SEED)
    pts += [tuple(int(v) for v in (rng.integers(0, nx), rng.integers(0, ny))) for _ in range(16)]
    return pts


def read_populations(s, form, pts):
    """f at the sampled nodes, from the current storage buffer [ny][9][pitch]:
    the state f_i(x) of a pull step is stored at x - v_i (include/kbc.h)."""
    buf = s.state_buffer()
    ny, nx = s.ny, s.nx
    x = np.array([p[0] for p in pts])[:, None]
    y = np.array([p[1] for p in pts])[:, None]
    ix = torch.as_tensor((x - CX[None, :]) % nx, device=buf.device)
    iy = torch.as_tensor((y - CY[None, :]) % ny, device=buf.device)
    ii = torch.as_tensor(np.broadcast_to(np.arange(9)[None, :], ix.shape).copy(), device=buf.device)
    v = buf[iy, ii, ix].double().cpu().numpy()      # [samples, 9]
    if form == "f16":
        v = v / (2.0 ** SHIFT)
    return v + W


def oracle_window(orc, ux, uy, beta, x, y, nsteps, storage=None):
    """f^nsteps at (x, y) from the oracle on a periodic window of half-width
    nsteps + 2 around (x, y): after n steps a node depends on the initial
    velocity within distance n + 1 (n streaming steps and the central
    differences of Grad's state), and the window's own wrap-around reaches
    inward one node per step, so its centre is exact."""
    ny, nx = ux.shape
    h = nsteps + 2
    d = np.arange(-h, h + 1)
    iy = torch.as_tensor((y + d) % ny, device=ux.device)[:, None]
    ix = torch.as_tensor((x + d) % nx, device=ux.device)[None, :]
    pu = np.ascontiguousarray(ux[iy, ix].cpu().numpy())
    pv = np.ascontiguousarray(uy[iy, ix].cpu().numpy())
    p = orc.Params(2 * h + 1, 2 * h + 1, beta, collision=orc.KBC, variant=orc.VARIANTS["B"], threads=4)
    f0 = orc.init(p, pu, pv)
    if storage is not None:
        f0 = orc.round_storage(p, f0, storage)
    f = orc.run(p, f0, nsteps, storage=storage)
    return f[:, h, h]


def check(orc, s, form, ux, uy, beta, pts, nsteps, tol):
    fg = read_populations(s, form, pts)
    fo = np.array([oracle_window(orc, ux, uy, beta, x, y, nsteps) for x, y in pts])
    fs = np.array([oracle_window(orc, ux, uy, beta, x, y, nsteps, storage=form) for x, y in pts])
    scale = np.abs(fo - W).max()
    sens = np.abs(fs - fo).max() / scale
    bar = max(tol, K_SENS * sens)
    err = np.abs(fg - fo).max() / scale
    worst = pts[int(np.abs(fg - fo).max(axis=1).argmax())]
    say(f"  {form} after {nsteps} step(s): {len(pts)} samples, err {err:.3e} at {worst}, "
        f"storage sensitivity {sens:.3e}, bar {bar:.3e}")
    assert np.isfinite(fg).all()
    assert err < bar


@pytest.mark.parametrize("form", ["f16", "f32"])
def test_storage_reader_matches_export(form):
    """The sampled reader above against the library's own FP64 export
    (lbm_get_populations) on a small ragged lattice after three steps."""
    nx, ny = 150, 70
    ux, uy = inputs.uniform_noise(nx, ny, AMP, SEED, "cuda")
    s = Sim(nx, ny, beta_from_nu(NU), collision="kbc", variant="B", form=form).init(ux, uy)
    s.step(3)
    pts = [(0, 0), (nx - 1, ny - 1), (0, ny - 1), (nx - 1, 0), (64, 16), (77, 33)]
    got = read_populations(s, form, pts)
    f = s.get_populations().cpu().numpy()
    want = np.array([f[:, y, x] for x, y in pts])
    assert np.abs(got - want).max() <= 1e-15


@pytest.mark.parametrize("form,n", [("f16", 65536), ("f32", 46400)])
def test_lattice_at_memory_limit(orc, form, n):
    nodes = n * n
    buf_bytes = 9 * n * n * STORE_BYTES[form]     # n is a multiple of 64: pitch = n
    need = 2 * buf_bytes + 2 * 8 * nodes + (4 << 30)
    torch.cuda.empty_cache()
    free, total = torch.cuda.mem_get_info()
    if free < need:
        pytest.skip(f"needs {need / 1e9:.0f} GB of device memory, {free / 1e9:.0f} GB free")
    say(f"max-size lattice {form} {n} x {n}: {nodes} nodes, two {buf_bytes / 1e9:.1f} GB buffers")
    beta = beta_from_nu(NU)
    ux, uy = inputs.uniform_noise(n, n, AMP, SEED, "cuda")
    s = Sim(n, n, beta, collision="kbc", variant="B", form=form, fusion=(1, 0)).init(ux, uy)
    assert s.pitch == n
    pts = sample_nodes(n, n, s.pitch, STORE_BYTES[form])
    say(f"  single step ({len(pts)} samples)")
    s.step(1)
    torch.cuda.synchronize()
    check(orc, s, form, ux, uy, beta, pts, 1, TOL1[form])
    s.set_fusion(2)
    say(f"  two fused steps, {s.fusion_rows}-row tiles")
    s.step(2)
    torch.cuda.synchronize()
    assert s.steps == 3
    check(orc, s, form, ux, uy, beta, pts, 3, TOL3[form])
    s.free()
    del s, ux, uy
    torch.cuda.empty_cache()


@pytest.mark.parametrize("nx,ny", [(64, 300000), (1048579, 3)])
def test_extreme_aspect_ratios(orc, nx, ny):
    """A tall lattice (300000 rows: the node kernels' grids run 75000
    workgroups in y) and a wide one (2^20 + 3 columns, the minimum 3 rows),
    FP32 KBC-B: one single step and two fused, sampled against oracle
    windows; then the moments (lbm_moments) at the same nodes against the
    oracle's moments of its window."""
    form = "f32"
    say(f"aspect {nx} x {ny}")
    beta = beta_from_nu(NU)
    ux, uy = inputs.uniform_noise(nx, ny, AMP, SEED, "cuda")
    s = Sim(nx, ny, beta, collision="kbc", variant="B", form=form, fusion=(1, 0)).init(ux, uy)
    rows = sorted({0, 1, 2, ny // 2, ny - 2, ny - 1, min(ny - 1, 4 * 65536), min(ny - 1, 4 * 65536 + 3)})
    cols = sorted(c for c in {0, 1, 63, 64, nx // 2, nx - 2, nx - 1} if c < nx)
    pts = [(x, y) for y in rows for x in cols]
    s.step(1)
    torch.cuda.synchronize()
    check(orc, s, form, ux, uy, beta, pts, 1, TOL1[form])
    s.set_fusion(2)
    s.step(2)
    torch.cuda.synchronize()
    check(orc, s, form, ux, uy, beta, pts, 3, TOL3[form])
    rho, mx, my = s.moments()
    xs = torch.as_tensor([p[0] for p in pts], device="cuda")
    ys = torch.as_tensor([p[1] for p in pts], device="cuda")
    got = np.stack([t[ys, xs].cpu().numpy() for t in (rho, mx, my)], axis=1)
    want = []
    for x, y in pts:
        h = 5
        d = np.arange(-h, h + 1)
        iy = torch.as_tensor((y + d) % ny, device="cuda")[:, None]
        ix = torch.as_tensor((x + d) % nx, device="cuda")[None, :]
        p = orc.Params(2 * h + 1, 2 * h + 1, beta, collision=orc.KBC, variant=orc.VARIANTS["B"])
        f = orc.run(p, orc.init(p, ux[iy, ix].cpu().numpy(), uy[iy, ix].cpu().numpy()), 3)
        r, u, v = orc.moments(p, f)
        want.append([r[h, h], u[h, h], v[h, h]])
    want = np.array(want)
    err_rho = np.abs(got[:, 0] - want[:, 0]).max()
    err_u = np.abs(got[:, 1:] - want[:, 1:]).max() / np.abs(want[:, 1:]).max()
    say(f"  moments after 3 steps: |drho| {err_rho:.2e}, u relative {err_u:.2e}")
    assert err_rho < 1e-6 and err_u < 1e-4
