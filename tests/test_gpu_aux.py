"""Checkpoint/resume of the image accumulation and the workspace poison mode, on the GPU.

Algorithm 1 adds each instance's level images to a running sum and stores the
sum once the instances are used up.  The running sum is a caller-owned float32
buffer and every call reads it and adds its own contribution in a fixed order,
so a run may stop after any call, store the buffer, and go on in another handle
from the stored values: the images come out bitwise the same as those of the
run that never stopped.

With BB_DEBUG_FILL=1 the library fills every workspace it is given with 0xFF
bytes (a NaN in float32 and float64) before it uses it; a read of workspace
memory that no kernel wrote would then change the results.  Every entry point
of standard synthesis gives bitwise the results it gives without the fill; the
NUFFT, whose grid points are added with FP32 atomics in an order that varies
between runs, gives finite images within 1e-6 of each level's peak of them.
"""

import sys

import numpy as np
import pytest
import torch

import oracle as ref
import sims
from oracle import levels_ref as lv
from oracle import nufft_ref as nf
from sims import configs
from tests._helpers import eig_inputs, level_errors, oracle_images

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


def _c4_items(n_side=40):
    w = configs.c4(n_channels=3, n_steps=4, n_side=n_side)
    items = []
    for i in range(w.n_instances()):
        inst = w.instance(i)
        items.append((inst.slot, inst.x, inst.wl, inst.W, inst.lam, inst.level_of))
    return w, items


@pytest.mark.parametrize("precision", ["fp32_3m", "bf16x3_3m"])
def test_checkpoint_resume_is_bitwise(ctx, tmp_path, precision):
    """The instances of a run in four calls (batched and single), once in one
    handle and once stopped after two calls: images and count stored to disk,
    the handle closed, a new handle created over the loaded images with the
    stored count, the last two calls made there.  Images and count bitwise equal;
    the whole against the oracle's sum over the instances."""
    from paper_2310_09200_amd import Batch, StandardSynthesis
    say(f"case checkpoint/resume precision={precision}")
    w, items = _c4_items()
    chunks = [items[0:5], items[5:6], items[6:10], items[10:]]

    def run(s, part):
        if len(part) == 1:
            sl, x, wl, W, d, lev = part[0]
            s.collect_eig(sl, x, wl, W, d, lev)
        else:
            s.collect_eig_batched(Batch(part, ctx.device))

    full = StandardSynthesis(ctx, w.pix, 4, 3, 512, 128, precision)
    for part in chunks:
        run(full, part)
    full.sync()
    want_img, want_count = full.images.cpu().numpy(), full.count
    full.close()

    a = StandardSynthesis(ctx, w.pix, 4, 3, 512, 128, precision)
    for part in chunks[:2]:
        run(a, part)
    a.sync()
    np.save(tmp_path / "images.npy", a.images.cpu().numpy())
    (tmp_path / "count.txt").write_text(str(a.count))
    a.close()

    restored = torch.from_numpy(np.load(tmp_path / "images.npy")).to(ctx.device)
    b = StandardSynthesis(ctx, w.pix, 4, 3, 512, 128, precision, images=restored)
    b.count = int((tmp_path / "count.txt").read_text())
    for part in chunks[2:]:
        run(b, part)
    b.sync()
    got_img, got_count = b.images.cpu().numpy(), b.count
    b.close()
    say(f"resumed vs uninterrupted: {np.count_nonzero(got_img != want_img)} differing values, "
        f"count {got_count} vs {want_count}")
    assert got_count == want_count == len(items)
    assert np.array_equal(got_img, want_img)
    want = np.zeros((3, 4, w.n_pix))
    for sl, x, wl, W, d, lev in items:
        Wc = W.astype(np.complex64).astype(np.complex128)
        want[sl] += oracle_images(Wc, d.astype(np.float32), lev, x, wl, w.pix, 4)
    tol = 1e-5 if precision == "fp32_3m" else 1e-4
    for sl in range(3):
        assert np.all(level_errors(got_img[sl], want[sl])[:, 0] <= tol), sl


def _standard_paths(ctx):
    """Every standard-synthesis entry point that takes or holds a workspace, on small inputs."""
    from paper_2310_09200_amd import Batch, StandardSynthesis
    out = {}
    w = configs.c1(n_ant=48, n_side=40)
    inst = w.instance(0)
    lam, W, iv, lev = eig_inputs(inst.V, inst.x, inst.wl, 40, 3)

    s = StandardSynthesis(ctx, w.pix, 4, 1, 48, 48, "fp32_3m")
    s.sync()
    ws = s.workspace.cpu().numpy()
    out["poisoned_fraction"] = np.array([np.mean(ws == 255)])
    s.collect_eig(0, inst.x, inst.wl, W, lam, lev)
    s.collect(0, inst.x, inst.wl, inst.V, 40, iv)
    s.sync()
    out["single+full"] = s.images.cpu().numpy()
    Wp, lamp, dp, levp = s.prestep(inst.x, inst.wl, inst.V, 40, iv)
    s.sync()
    out["prestep"] = np.concatenate([lamp.cpu().numpy().view(np.uint8), dp.cpu().numpy().view(np.uint8),
                                     levp.cpu().numpy().view(np.uint8)])
    xs = np.stack([sims.earth_rotate(inst.x, 0.3 * i) for i in range(3)])
    Wb, lamb, db, levb = s.prestep_batched(xs, [inst.wl] * 3, np.stack([inst.V] * 3), 40, iv)
    s.sync()
    out["prestep_batched"] = np.concatenate([lamb.cpu().numpy().ravel().view(np.uint8),
                                             levb.cpu().numpy().ravel().view(np.uint8)])
    s.reset()
    s.collect_eig_batched(Batch([(0, xs[i], inst.wl, Wb[i], db[i], levb[i]) for i in range(3)], ctx.device))
    s.sync()
    out["batched"] = s.images.cpu().numpy()
    g = np.random.default_rng(3).normal(size=(4, w.n_pix))
    dW, dd, dx = s.eig_backward(inst.x, inst.wl, W, lam, lev, g)
    s.sync()
    out["backward"] = np.concatenate([dW.cpu().numpy().ravel().view(np.uint8), dd.cpu().numpy().view(np.uint8),
                                      dx.cpu().numpy().ravel().view(np.uint8)])
    s.close()

    wb, items = _c4_items(n_side=24)
    s = StandardSynthesis(ctx, wb.pix, 4, 3, 512, 128, "bf16x3_3m")
    s.collect_eig_batched(Batch(items, ctx.device))
    s.sync()
    out["batched_bf16"] = s.images.cpu().numpy()
    s.close()
    return out


def _nufft_paths(ctx):
    """NUFFT synthesis: one plan, and one split into image tiles and uvw cells."""
    from paper_2310_09200_amd import Batch, NufftSynthesis
    out = {}
    w = configs.c1(n_ant=48, n_side=36, fov_deg=10.0)
    inst = w.instance(0)
    items = []
    for i, L in enumerate([48, 40]):
        x = sims.earth_rotate(inst.x[:L], 0.3 * i)
        lam, A = ref.geneig(inst.V[:L, :L], ref.gram(x, inst.wl))
        lam, W = ref.select_top(lam, A, 32)
        items.append((x, inst.wl, W, lam))
    iv = lv.kmeans_intervals(np.concatenate([it[3] for it in items]), 3)
    frame = np.array(sims.tangent_basis(90.0))
    uvw = np.zeros(3)
    for x, wl, _, _ in items:
        li, mi = np.triu_indices(x.shape[0], k=1)
        uvw = np.maximum(uvw, np.max(np.abs(nf.rotate(x[li] - x[mi], frame) / wl), axis=0))
    uvw = np.maximum(uvw * 1.01, 1.0)
    n_levels = iv.shape[0]
    batch = Batch([(0, x, wl, W, ref.lsq_filter(lam), lv.level_of(lam, iv)) for x, wl, W, lam in items], ctx.device)
    for name, P, Q in [("nufft", 1, 1), ("nufft_partitioned", 2, 2)]:
        plan = NufftSynthesis(ctx, w.pix, n_levels, 64, 64, 1e-5, frame, uvw, partitions=P, uvw_partitions=Q)
        plan.collect_eig_batched(batch)
        plan.emit()
        plan.collect_eig_batched(batch)
        plan.emit()
        plan.sync()
        out[name] = plan.images.cpu().numpy()
        plan.close()
    return out


def test_debug_fill_leaves_every_result_unchanged(ctx, monkeypatch):
    """Each entry point run twice, without and with BB_DEBUG_FILL=1: bitwise the
    same images, eigenvalues, weights, level ids and gradients (NUFFT images
    within the run-to-run spread of their atomic sums); the handle's
    workspace after create holds the 0xFF fill (apart from the few words create
    itself writes) in the second run."""
    say("case BB_DEBUG_FILL: standard synthesis entry points and NUFFT plans")
    monkeypatch.delenv("BB_DEBUG_FILL", raising=False)
    plain = {**_standard_paths(ctx), **_nufft_paths(ctx)}
    monkeypatch.setenv("BB_DEBUG_FILL", "1")
    poisoned = {**_standard_paths(ctx), **_nufft_paths(ctx)}
    monkeypatch.delenv("BB_DEBUG_FILL")
    say(f"workspace fill fraction after create: {plain['poisoned_fraction'][0]:.4f} plain, "
        f"{poisoned['poisoned_fraction'][0]:.4f} with BB_DEBUG_FILL")
    assert poisoned["poisoned_fraction"][0] > 0.9
    for k in plain:
        if k == "poisoned_fraction":
            continue
        if plain[k].dtype == np.float32:
            assert np.all(np.isfinite(plain[k])) and np.all(np.isfinite(poisoned[k])), k
        if k.startswith("nufft"):
            # grid points added with FP32 atomics: the last bits vary between runs
            rel = np.max(np.abs(plain[k] - poisoned[k]), axis=-1) / np.max(np.abs(plain[k]), axis=-1)
            say(f"{k}: max difference per level / level peak {np.array2string(rel, precision=2)}")
            assert np.all(rel <= 1e-6), k
            continue
        same = np.array_equal(plain[k], poisoned[k])
        say(f"{k}: {'bitwise equal' if same else 'DIFFERS'}")
        assert same, k


def test_tune_cache_written_by_autotune_and_read_by_create(ctx, tmp_path, monkeypatch):
    """BB_TUNE_CACHE: a handle starts from the cached tiles of its key; autotuning
    replaces the entries of the classes it timed (other lines kept) and a new
    handle then starts from the tuned tiles; an unwritable cache fails the
    autotune call with BB_ERR_STATE while the handle keeps its tuned tiles."""
    import json

    from paper_2310_09200_amd import Batch, BluebildError, StandardSynthesis, _lib, tile_shapes
    say("case autotune cache")
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    g = np.random.default_rng(12)
    pix = sims.pixel_grid(40, 6.0, 60.0)          # 1600 pixels: pix_log2 = 10
    wl = sims.wavelength_m(150e6)
    items = []
    for i, (L, K) in enumerate([(60, 20), (70, 50), (80, 100)]):
        x = sims.disk_layout(L, 3000.0, g, z_sigma_m=2.0)
        items.append((0, x, wl, sims.random_eigvecs(L, K, g).astype(np.complex64),
                      g.normal(0, 1, K).astype(np.float32), g.integers(0, 2, K).astype(np.int32)))
    path = tmp_path / "tune.jsonl"
    other = '{"arch": "%s", "precision": 2, "k_class": 2, "pix_log2": 11, "tile": 1, "ms": 1.0}' % arch
    path.write_text('{"arch": "%s", "precision": 2, "k_class": 2, "pix_log2": 10, "tile": 6, "ms": 5.0}\n'
                    'kept as it is\n%s\n' % (arch, other))
    monkeypatch.setenv("BB_TUNE_CACHE", str(path))
    s = StandardSynthesis(ctx, pix, 2, 1, 80, 100, "fp32_3m")
    assert s.tiles == [3, 9, 6, 0]                # class 2 from the cache, the rest defaults
    ms = s.autotune_batched(Batch(items, ctx.device), reps=1)
    s.sync()
    tuned = s.tiles
    s.close()
    lines = path.read_text().splitlines()
    assert "kept as it is" in lines and other in lines
    entries = [json.loads(ln) for ln in lines if ln.startswith("{") and ln != other]
    assert sorted(e["k_class"] for e in entries) == sorted(ms)
    for e in entries:
        assert (e["arch"], e["precision"], e["pix_log2"]) == (arch, 2, 10)
        assert e["tile"] == tuned[e["k_class"]] and e["ms"] == pytest.approx(ms[e["k_class"]][e["tile"]], abs=1e-3)
    s2 = StandardSynthesis(ctx, pix, 2, 1, 80, 100, "fp32_3m")
    assert s2.tiles == tuned
    s2.close()
    s3 = StandardSynthesis(ctx, pix[:1000], 2, 1, 80, 100, "fp32_3m")   # another pixel key: defaults
    assert s3.tiles == [3, 9, 11, 0]
    s3.close()
    monkeypatch.setenv("BB_TUNE_CACHE", str(tmp_path / "no_such_dir" / "tune.jsonl"))
    s4 = StandardSynthesis(ctx, pix, 2, 1, 80, 100, "fp32_3m")
    s4.tiles = [3, 2, 1, 0]
    with pytest.raises(BluebildError) as e:
        s4.autotune_batched(Batch(items, ctx.device), reps=1)
    assert e.value.status == _lib.BB_ERR_STATE
    shapes = tile_shapes("fp32_3m")
    for c in range(3):                            # tuned: a candidate of each timed class
        assert c in next(cl for t, *_, cl in shapes if t == s4.tiles[c])
    assert s4.tiles[3] == 0                       # class 3 was not in the batch
    s4.close()
