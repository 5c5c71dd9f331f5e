"""GPU NUFFT synthesis against the oracle (through the C ABI).

The gate: the NUFFT's accuracy contract against the exact image (standard
synthesis of the same eigenpairs, Section 2.4): per level
|I - I_exact| <= 2 eps sum_{q<r} |V'[r, q]| (Section 3.4), independent of
any convention of the transform's steps.  Beside it, the oracle's NUFFT (the
same steps and constants in FP64, with the oracle's stated convention for
kernel windows on exact ties): the GPU's FP32 grid and transform agree with
it to about 1e-5 of each level's peak.
"""

import sys

import numpy as np
import pytest

import oracle as ref
import sims
from oracle import levels_ref as lv
from oracle import nufft_ref as nf
from sims import configs

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx(gpu):
    from paper_2310_09200_amd import Context
    c = Context(0)
    yield c
    c.close()


def _instances(n_inst, n_ant, n_side, n_pos, seed, fov_deg=5.0):
    """Eigenpairs of C1-like instances (array rotated per instance), all positive levels + 1 negative."""
    w = configs.c1(n_ant=max(n_ant), n_side=n_side, fov_deg=fov_deg)
    g = sims.rng(95, seed)
    out = []
    for i in range(n_inst):
        inst = w.instance(0)
        L = n_ant[i % len(n_ant)]
        x = sims.earth_rotate(inst.x[:L], 0.3 * i)
        V = inst.V[:L, :L]
        wl = inst.wl * (1.0 + 0.1 * i)
        lam, A = ref.geneig(V, ref.gram(x, wl))
        K = min(L, 40)
        lam, W = ref.select_top(lam, A, K)
        out.append((x, wl, W, lam))
    lam_all = np.concatenate([o[3] for o in out])
    iv = lv.kmeans_intervals(lam_all, n_pos)
    items = []
    for x, wl, W, lam in out:
        items.append((x, wl, W, ref.lsq_filter(lam), ref.level_membership(lam, iv), lv.level_of(lam, iv)))
    return w.pix, items, iv.shape[0]


def _uvw_bound(items, frame):
    b = np.zeros(3)
    for x, wl, *_ in items:
        li, mi = np.triu_indices(x.shape[0], k=1)
        b = np.maximum(b, np.max(np.abs(nf.rotate(x[li] - x[mi], frame) / wl), axis=0))
    return b * 1.01


def _run(ctx, pix, items, n_levels, eps, frame, uvw, n_ant_max=64, k_max=64, emits=1, transform="auto"):
    from paper_2310_09200_amd import Batch, NufftSynthesis
    plan = NufftSynthesis(ctx, pix, n_levels, n_ant_max, k_max, eps, frame, uvw, transform=transform)
    chunks = np.array_split(np.arange(len(items)), emits)
    for ch in chunks:
        b = Batch([(0, items[i][0], items[i][1], items[i][2], items[i][3], items[i][5]) for i in ch], ctx.device)
        plan.collect_eig_batched(b)
        plan.emit()
    plan.sync()
    got = plan.images.double().cpu().numpy()
    shape = plan.shape
    plan.close()
    return got, shape


def _check(got, want, tol):
    for a, b in zip(got, want):
        peak = np.max(np.abs(b))
        assert np.max(np.abs(a - b)) <= tol * peak, (np.max(np.abs(a - b)) / peak, tol)


def _check_contract(got, want, insts, eps):
    """The NUFFT's accuracy contract: per level, |I - I_exact| <= 2 eps sum_{q<r} |V'[r, q]|
    (the image is 2 Re of the transformed sum), plus FP32 slack of 1e-5 of the peak."""
    l1 = 0.0
    for x, wl, W, d, member in insts:
        Vp = nf.level_visibilities(W, d, member)
        li, mi = np.triu_indices(x.shape[0], k=1)
        l1 = l1 + np.abs(Vp[:, mi, li]).sum(axis=1)
    for lv, (a, b) in enumerate(zip(got, want)):
        err = np.max(np.abs(a - b))
        assert err <= 2 * eps * l1[lv] + 1e-5 * np.max(np.abs(b)), (lv, err, 2 * eps * l1[lv])


@pytest.mark.parametrize("eps", [1e-3, 1e-5, 1e-6])
def test_nufft_single_instance(ctx, eps):
    say(f"case nufft single instance eps={eps}")
    pix, items, n_levels = _instances(1, [48], 40, 3, 0)
    frame = np.array(sims.tangent_basis(90.0))
    uvw = _uvw_bound(items, frame)
    got, (N, M, w) = _run(ctx, pix, items, n_levels, eps, frame, uvw)
    P = nf.plan_params(eps, uvw, nf.rotate(pix, frame))
    assert list(N) == list(P["N"]) and list(M) == list(P["M"]) and w == P["w"]
    want_nufft = nf.nufft_images([(x, wl, W, d, mem) for x, wl, W, d, mem, _ in items], pix, eps, X=uvw, frame=frame)
    _check(got, want_nufft, 1e-5)
    x, wl, W, d, mem, _ = items[0]
    want = ref.synthesize_blas(W, d, mem, x, pix, wl)
    _check_contract(got, want, [(x, wl, W, d, mem)], eps)
    _check(got, want, 3 * eps + 1e-5)


def test_nufft_batched_ragged_instances(ctx):
    say("case nufft three instances, L = 48 / 37 / 64, two emits")
    pix, items, n_levels = _instances(3, [48, 37, 64], 32, 4, 1)
    frame = np.array(sims.tangent_basis(90.0))
    uvw = _uvw_bound(items, frame)
    got, _ = _run(ctx, pix, items, n_levels, 1e-5, frame, uvw, emits=2)
    want = sum(ref.synthesize_blas(W, d, mem, x, pix, wl) for x, wl, W, d, mem, _ in items)
    _check_contract(got, want, [(x, wl, W, d, mem) for x, wl, W, d, mem, _ in items], 1e-5)
    _check(got, want, 4e-5)
    want_nufft = nf.nufft_images([(x, wl, W, d, mem) for x, wl, W, d, mem, _ in items], pix, 1e-5, X=uvw, frame=frame)
    _check(got, want_nufft, 1e-5)


@pytest.mark.parametrize("eps", [1e-4, 1e-6])
def test_nufft_transforms_agree(ctx, eps):
    """The library's own line FFTs and rocFFT compute the same pruned transform:
    both within 1e-5 of the FP64 NUFFT oracle and within FP32 rounding of each other."""
    say(f"case nufft line FFTs vs rocFFT, eps={eps}")
    pix, items, n_levels = _instances(3, [48, 37, 64], 32, 4, 3)
    frame = np.array(sims.tangent_basis(90.0))
    uvw = _uvw_bound(items, frame)
    got_line, _ = _run(ctx, pix, items, n_levels, eps, frame, uvw, transform="auto")
    got_roc, _ = _run(ctx, pix, items, n_levels, eps, frame, uvw, transform="rocfft")
    want_nufft = nf.nufft_images([(x, wl, W, d, mem) for x, wl, W, d, mem, _ in items], pix, eps, X=uvw, frame=frame)
    _check(got_line, want_nufft, 1e-5)
    _check(got_roc, want_nufft, 1e-5)
    _check(got_line, got_roc, 5e-6)
    insts = [(x, wl, W, d, mem) for x, wl, W, d, mem, _ in items]
    want = sum(ref.synthesize_blas(W, d, mem, x, pix, wl) for x, wl, W, d, mem in insts)
    _check_contract(got_line, want, insts, eps)
    _check_contract(got_roc, want, insts, eps)


def test_nufft_tilted_frame(ctx):
    """Pixels around a phase centre at declination +50 deg; the grid is thin along p0."""
    say("case nufft tilted frame")
    w = configs.c1(n_ant=40, n_side=24)
    inst = w.instance(0)
    pix = sims.pixel_grid(24, 4.0, 50.0)
    frame = np.array(sims.tangent_basis(50.0))
    lam, A = ref.geneig(inst.V, ref.gram(inst.x, inst.wl))
    lam, W = ref.select_top(lam, A, 40)
    iv = lv.kmeans_intervals(lam, 2)
    items = [(inst.x, inst.wl, W, ref.lsq_filter(lam), ref.level_membership(lam, iv), lv.level_of(lam, iv))]
    uvw = _uvw_bound(items, frame)
    got, (N, M, wk) = _run(ctx, pix, items, iv.shape[0], 1e-5, frame, uvw)
    assert N[2] < N[0]
    want = ref.synthesize_blas(W, ref.lsq_filter(lam), items[0][4], inst.x, pix, inst.wl)
    _check_contract(got, want, [(inst.x, inst.wl, W, ref.lsq_filter(lam), items[0][4])], 1e-5)
    _check(got, want, 4e-5)


def test_nufft_baseline_beyond_bound_reported(ctx):
    from paper_2310_09200_amd import Batch, BluebildError, NufftSynthesis
    say("case nufft baseline beyond uvw_max")
    pix, items, n_levels = _instances(1, [16], 16, 2, 2)
    frame = np.eye(3)
    uvw = np.maximum(_uvw_bound(items, frame) * 0.5, 1.0)   # the flat array has no extent along z
    plan = NufftSynthesis(ctx, pix, n_levels, 16, 16, 1e-4, frame, uvw)
    x, wl, W, d, mem, lev = items[0]
    plan.collect_eig_batched(Batch([(0, x, wl, W, d, lev)], ctx.device))
    plan.emit()
    with pytest.raises(BluebildError, match="uvw_max"):
        plan.sync()
    assert np.all(np.isfinite(plan.images.cpu().numpy()))
    plan.close()


def test_nufft_rejects_bad_options(ctx):
    from paper_2310_09200_amd import BluebildError, NufftSynthesis
    pix = sims.pixel_grid(8, 2.0)
    with pytest.raises(BluebildError):
        NufftSynthesis(ctx, pix, 2, 16, 16, 1e-9, np.eye(3), [10.0, 10.0, 10.0])
    with pytest.raises(BluebildError):
        NufftSynthesis(ctx, pix, 2, 16, 16, 1e-4, np.diag([1.0, 1.0, 2.0]), [10.0, 10.0, 10.0])
    from paper_2310_09200_amd import _lib
    opt = _lib.bb_nufft_options(n_levels=2, n_ant_max=16, k_max=16, transform=2, epsilon=1e-4)
    opt.frame[0] = opt.frame[4] = opt.frame[8] = 1.0
    for i in range(3):
        opt.uvw_max[i] = 10.0
    pix_cm = np.ascontiguousarray(np.asarray(pix, np.float64).T)
    import ctypes
    sz = ctypes.c_size_t()
    assert ctx.lib.bb_nufft_workspace_size(ctx.handle, ctypes.byref(opt), pix_cm.shape[1],
                                           ctypes.c_void_p(pix_cm.ctypes.data), ctypes.byref(sz)) != 0


@pytest.mark.parametrize("transform", ["auto", "rocfft"])
@pytest.mark.parametrize("fov_deg,path", [(20.0, "output-driven, two rows per column"),
                                          (30.0, "output-driven, four rows per column"),
                                          (45.0, "tiles of 8 grid points"), (60.0, "global atomics")])
def test_nufft_thick_grids(ctx, fov_deg, path, transform):
    """A 3-D antenna cloud and a wide field make the grid thick along p0: the
    output-driven spread with 32 or 64 lanes per column (16 < N2 <= 64), LDS
    tiles of 8 points (64 < N2 <= 128) or, past 128 points, global atomics;
    against standard synthesis."""
    from paper_2310_09200_amd import Batch, NufftSynthesis
    say(f"case nufft thick grid, field {fov_deg} deg ({path}), transform {transform}")
    g = sims.rng(96, int(fov_deg))
    L, K = 40, 20
    x = g.uniform(-150.0, 150.0, (L, 3))
    wl = 2.0
    pix = sims.pixel_grid(16, fov_deg, 90.0)
    W = (g.normal(size=(L, K)) + 1j * g.normal(size=(L, K))) / np.sqrt(2 * L)
    d = np.exp(g.normal(size=K)) * np.where(np.arange(K) < 15, 1.0, -1.0)
    lev = np.minimum(np.arange(K) // 6, 2).astype(np.int32)
    member = ref.membership_from_level_of(lev, 3)
    frame = np.array(sims.tangent_basis(90.0))
    items = [(x, wl, W, d, member, lev)]
    uvw = _uvw_bound(items, frame)
    eps = 1e-4
    plan = NufftSynthesis(ctx, pix, 3, L, K, eps, frame, uvw, transform=transform)
    N, M, wk = plan.shape
    assert {20.0: 16 < N[2] <= 32, 30.0: 32 < N[2] <= 64, 45.0: 64 < N[2] <= 128, 60.0: N[2] > 128}[fov_deg], N
    plan.collect_eig_batched(Batch([(0, x, wl, W, d, lev)], ctx.device))
    plan.emit()
    plan.sync()
    got = plan.images.double().cpu().numpy()
    plan.close()
    want = ref.synthesize_blas(W, d, member, x, pix, wl)
    _check_contract(got, want, [(x, wl, W, d, member)], eps)
    if fov_deg <= 30.0:  # small enough for the FP64 NUFFT oracle on the host
        want_nufft = nf.nufft_images([(x, wl, W, d, member)], pix, eps, X=uvw, frame=frame)
        _check(got, want_nufft, 1e-5)


def test_nufft_dense_uv_split_parts(ctx):
    """Many epochs of a compact array pile baselines into few grid columns, so
    the output-driven spread splits busy column blocks into parts added with
    atomics (a column sees more than 4096 baselines); against the FP64 NUFFT
    oracle and standard synthesis."""
    from paper_2310_09200_amd import Batch, NufftSynthesis
    say("case nufft dense uv plane: split column blocks")
    g = sims.rng(97, 0)
    L, K, n_ep = 64, 24, 12
    base = g.uniform(-40.0, 40.0, (L, 3))
    base[:, 2] = 0.0
    wl = 2.0
    pix = sims.pixel_grid(20, 6.0, 90.0)
    frame = np.array(sims.tangent_basis(90.0))
    items = []
    for e in range(n_ep):
        x = sims.earth_rotate(base, 0.02 * e)
        W = (g.normal(size=(L, K)) + 1j * g.normal(size=(L, K))) / np.sqrt(2 * L)
        d = np.exp(g.normal(size=K))
        lev = np.minimum(np.arange(K) // 8, 2).astype(np.int32)
        items.append((x, wl, W, d, ref.membership_from_level_of(lev, 3), lev))
    uvw = np.maximum(_uvw_bound(items, frame), 1.0)  # the array is flat: no extent along p0
    eps = 1e-4
    # the busiest grid column must see more than 4096 baselines
    P = nf.plan_params(eps, uvw, nf.rotate(pix, frame))
    N, h, wk = P["N"], P["h"], P["w"]
    cnt = np.zeros((N[0], N[1]), np.int64)
    for x, wl_, *_ in items:
        li, mi = np.triu_indices(L, k=1)
        xi = nf.rotate(x[li] - x[mi], frame) / wl_ / h
        f0 = np.mod(np.ceil(xi[:, 0] - 0.5 * wk).astype(np.int64), N[0])
        f1 = np.mod(np.ceil(xi[:, 1] - 0.5 * wk).astype(np.int64), N[1])
        np.add.at(cnt, (f0, f1), 1)
    col = sum(np.roll(np.roll(cnt, a, axis=0), c, axis=1) for a in range(wk) for c in range(wk))
    assert col.max() > 4096, col.max()
    plan = NufftSynthesis(ctx, pix, 3, L, K, eps, frame, uvw)
    plan.collect_eig_batched(Batch([(0, x, wl_, W, d, lev) for x, wl_, W, d, _, lev in items], ctx.device))
    plan.emit()
    plan.sync()
    got = plan.images.double().cpu().numpy()
    plan.close()
    want_nufft = nf.nufft_images([(x, wl_, W, d, mem) for x, wl_, W, d, mem, _ in items], pix, eps, X=uvw, frame=frame)
    _check(got, want_nufft, 1e-5)
    want = sum(ref.synthesize_blas(W, d, mem, x, pix, wl_) for x, wl_, W, d, mem, _ in items)
    _check_contract(got, want, [(x, wl_, W, d, mem) for x, wl_, W, d, mem, _ in items], eps)


def _tiles(pix, frame, P):
    """Pixel indices of the nonempty P x P tiles of the field along e_u, e_v (the library's split)."""
    u = (pix[:, 0] * frame[0, 0] + pix[:, 1] * frame[0, 1]) + pix[:, 2] * frame[0, 2]
    v = (pix[:, 0] * frame[1, 0] + pix[:, 1] * frame[1, 1]) + pix[:, 2] * frame[1, 2]

    def cell(x):
        span = x.max() - x.min()
        if not span > 0:
            return np.zeros(x.shape, np.int64)
        return np.clip(((x - x.min()) / span * P).astype(np.int64), 0, P - 1)

    key = cell(u) * P + cell(v)
    return [np.nonzero(key == k)[0] for k in range(P * P) if np.any(key == k)]


@pytest.mark.parametrize("P", [2, 4])
def test_nufft_image_partitions(ctx, P):
    """Image-domain partitions: every tile of the field is its own NUFFT (grid
    sized to the tile); a cross of pixels leaves the corner tiles empty.  Each
    tile against the FP64 NUFFT oracle on its pixels, the whole against
    standard synthesis."""
    from paper_2310_09200_amd import Batch, NufftSynthesis
    say(f"case nufft image partitions {P} x {P}")
    pix_all, items, n_levels = _instances(2, [48, 40], 40, 3, 4, fov_deg=12.0)
    frame = np.array(sims.tangent_basis(90.0))
    uv = nf.rotate(pix_all, frame)[:, :2]
    half = np.abs(uv).max()
    pix = pix_all[(np.abs(uv[:, 0]) < 0.3 * half) | (np.abs(uv[:, 1]) < 0.3 * half)]
    uvw = np.maximum(_uvw_bound(items, frame), 1.0)
    eps = 1e-5
    plan = NufftSynthesis(ctx, pix, n_levels, 64, 64, eps, frame, uvw, partitions=P)
    plan_one = NufftSynthesis(ctx, pix, n_levels, 64, 64, eps, frame, uvw)
    assert np.prod(plan.shape[0]) < np.prod(plan_one.shape[0])
    plan_one.close()
    b = Batch([(0, x, wl, W, d, lev) for x, wl, W, d, _, lev in items], ctx.device)
    plan.collect_eig_batched(b)
    plan.emit()
    plan.sync()
    got = plan.images.double().cpu().numpy()
    plan.close()
    tiles = _tiles(pix, frame, P)
    assert sum(len(t) for t in tiles) == pix.shape[0] and len(tiles) == (P * P if P < 4 else P * P - 4)
    insts = [(x, wl, W, d, mem) for x, wl, W, d, mem, _ in items]
    for t in tiles:
        want_t = nf.nufft_images(insts, pix[t], eps, X=uvw, frame=frame)
        _check(got[:, t], want_t, 1e-5)
    want = sum(ref.synthesize_blas(W, d, mem, x, pix, wl) for x, wl, W, d, mem, _ in items)
    _check_contract(got, want, insts, eps)


@pytest.mark.parametrize("Q,P", [(2, 1), (3, 1), (2, 2)])
def test_nufft_uvw_partitions(ctx, Q, P):
    """uvw-domain partitions (Section 3.4.1): Q x Q cells of the baselines along
    e_u, e_v, each shifted by its centre and transformed on a grid sized by the
    cell (one NUFFT per (tile, cell), one after another on one shared grid).
    Against the FP64 oracle's cell-split NUFFT (the same steps) per image tile,
    and against standard synthesis within the accuracy contract; the images
    come from two collect calls (each transforms at once) and one emit."""
    from paper_2310_09200_amd import Batch, NufftSynthesis
    say(f"case nufft uvw partitions {Q} x {Q}, image partitions {P} x {P}")
    pix, items, n_levels = _instances(3, [48, 40, 44], 36, 3, 6, fov_deg=10.0)
    frame = np.array(sims.tangent_basis(90.0))
    uvw = np.maximum(_uvw_bound(items, frame), 1.0)
    eps = 1e-5
    plan = NufftSynthesis(ctx, pix, n_levels, 64, 64, eps, frame, uvw, partitions=P, uvw_partitions=Q)
    whole = NufftSynthesis(ctx, pix, n_levels, 64, 64, eps, frame, uvw)
    (N, _, _), (Nw, _, _) = plan.shape, whole.shape
    whole.close()
    if P == 1:
        assert N[0] < Nw[0] and N[1] < Nw[1], (N, Nw)
    b1 = Batch([(0, x, wl, W, d, lev) for x, wl, W, d, _, lev in items[:2]], ctx.device)
    b2 = Batch([(0, x, wl, W, d, lev) for x, wl, W, d, _, lev in items[2:]], ctx.device)
    plan.collect_eig_batched(b1)
    plan.collect_eig_batched(b2)
    plan.emit()
    plan.sync()
    got = plan.images.double().cpu().numpy()
    plan.close()
    insts = [(x, wl, W, d, mem) for x, wl, W, d, mem, _ in items]
    tiles = _tiles(pix, frame, P) if P > 1 else [np.arange(pix.shape[0])]
    for t in tiles:
        want_t = nf.nufft_images(insts, pix[t], eps, X=uvw, frame=frame, uvw_cells=Q)
        _check(got[:, t], want_t, 1e-5)
    want = sum(ref.synthesize_blas(W, d, mem, x, pix, wl) for x, wl, W, d, mem in insts)
    _check_contract(got, want, insts, eps)
