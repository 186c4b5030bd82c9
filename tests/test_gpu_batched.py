"""GPU: batched applies over plans of mixed d, N, kernel and k.

The batch runs stage by stage with grouped launches (one launch per stage and
kernel shape, workgroups taking (density, tile) items) captured in a HIP graph.
Every tile runs the same code as in a single-plan apply, so batched results
must equal single applies bit for bit; a sample of the mixed 64-density batch
is also checked against the FP64 oracle at the FP32 bar (relative L2 and
relative max error 1e-5).
"""
import sys

import numpy as np
import pytest

from parity import check  # noqa: E402

pytestmark = pytest.mark.gpu

FP32_TOL = 1e-5


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _vg():
    import paper_1604_03155_amd as vg
    return vg


def _torch():
    import torch
    return torch




def random_density(seed, d, N):
    rng = np.random.default_rng(seed)
    return (rng.standard_normal((N,) * d) + 1j * rng.standard_normal((N,) * d)).astype(np.complex128)


def dev(f, precision="fp32"):
    torch = _torch()
    dt = torch.complex128 if precision == "fp64" else torch.complex64
    return torch.from_numpy(f).to(dtype=dt, device="cuda").contiguous()


@pytest.fixture(scope="module")
def c4():
    """The 64-density mixed batch (N in {48, 64, 96, 128}, Laplace and
    Helmholtz k ~ U[5, 40]) with FP32 plans and its densities on the device."""
    from workloads import batch_workload, evaluate_grid
    vg = _vg()
    items = batch_workload()
    plans, fs_host, fs = [], [], []
    for prm, src in items:
        plans.append(vg.Plan(3, prm["N"], prm["kernel"], prm["k"], precision="fp32"))
        f = evaluate_grid(src, prm["N"])
        fs_host.append(f)
        fs.append(dev(f))
    return items, plans, fs_host, fs


def singles(plans, fs):
    return [p.apply(f) for p, f in zip(plans, fs)]


def test_c4_batch_bitwise_equals_single_applies(c4):
    say("c4 bitwise")
    vg = _vg()
    torch = _torch()
    _, plans, _, fs = c4
    ref = singles(plans, fs)
    out = vg.apply_batched(plans, fs)
    torch.cuda.synchronize()
    for i, (a, b) in enumerate(zip(out, ref)):
        assert torch.equal(a, b), i


def test_c4_batch_sample_against_oracle(c4):
    """Two densities of every size (one Laplace, one Helmholtz where the draw
    has both) against the FP64 oracle."""
    say("c4 oracle sample")
    from oracle import operator as op
    vg = _vg()
    torch = _torch()
    items, plans, fs_host, fs = c4
    out = vg.apply_batched(plans, fs)
    torch.cuda.synchronize()
    picked = {}
    for i, (prm, _) in enumerate(items):
        key = (prm["N"], prm["kernel"])
        picked.setdefault(key, i)
    assert len(picked) == 8
    for (N, kernel), i in sorted(picked.items()):
        prm = items[i][0]
        say("  oracle", i, N, kernel, prm["k"])
        o = op.Plan(3, N, kernel, prm["k"])
        check(out[i].cpu().numpy(), o.apply(fs_host[i]), FP32_TOL, i)


def test_c4_graph_replays_track_new_density_values(c4):
    """Same arrays, new contents: the captured graph replays (with eager work
    and synchronisations in between) and every replay matches single applies."""
    say("c4 replays")
    vg = _vg()
    torch = _torch()
    _, plans, _, fs = c4
    work = [f.clone() for f in fs]
    outs = [torch.empty_like(f) for f in fs]
    for r in range(3):
        for j, w in enumerate(work):
            w.mul_(complex(0.5 + 0.25 * r, 0.1 * (j % 3)))
        scratch = torch.randn(1 << 20, device="cuda").sum()  # eager work between replays
        vg.apply_batched(plans, work, outs)
        torch.cuda.synchronize()
        assert torch.isfinite(scratch)
        ref = singles(plans, work)
        torch.cuda.synchronize()
        for i, (a, b) in enumerate(zip(outs, ref)):
            assert torch.equal(a, b), (r, i)


def test_c4_explicit_workspace_and_stream(c4):
    say("c4 workspace/stream")
    vg = _vg()
    torch = _torch()
    _, plans, _, fs = c4
    nbytes = vg.batched_workspace_size(plans)
    ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    s = torch.cuda.Stream()
    outs = [torch.empty_like(f) for f in fs]
    torch.cuda.synchronize()
    with torch.cuda.stream(s):
        vg.apply_batched(plans, fs, outs, workspace=ws, stream=s)
    s.synchronize()
    ref = singles(plans, fs)
    torch.cuda.synchronize()
    for i, (a, b) in enumerate(zip(outs, ref)):
        assert torch.equal(a, b), i


def test_batched_mixed_dimensions_and_ungrouped_paths(monkeypatch):
    """2D and 3D plans in one batch, duplicated sizes (grouped launches) and
    singletons; the same batch with grouping and graphs switched off agrees."""
    say("mixed d")
    vg = _vg()
    torch = _torch()
    specs = [(2, 64, "laplace", 0.0), (3, 32, "helmholtz", 9.0), (2, 64, "helmholtz", 10.0),
             (3, 32, "laplace", 0.0), (2, 48, "helmholtz", 3.0), (3, 24, "helmholtz", 4.0),
             (3, 32, "helmholtz", 12.0), (2, 64, "laplace", 0.0), (2, 512, "helmholtz", 40.0),
             (2, 512, "laplace", 0.0)]
    plans = [vg.Plan(d, N, kind, k, precision="fp32") for d, N, kind, k in specs]
    fs = [dev(random_density(50 + i, d, N)) for i, (d, N, _, _) in enumerate(specs)]
    ref = singles(plans, fs)
    out = vg.apply_batched(plans, fs)
    torch.cuda.synchronize()
    for i, (a, b) in enumerate(zip(out, ref)):
        assert torch.equal(a, b), i
    monkeypatch.setenv("VG_BATCH_NO_GROUP", "1")
    monkeypatch.setenv("VG_BATCH_NO_GRAPH", "1")
    out2 = vg.apply_batched(plans, fs)  # new output arrays: a new batch entry
    torch.cuda.synchronize()
    for i, (a, b) in enumerate(zip(out2, ref)):
        assert torch.equal(a, b), i


def test_batched_wide_column_tiles():
    """Two 3D N = 512 densities (plain column passes of length 1024 on 16-pencil
    tiles, grouped into one launch per stage) next to a small one: bitwise
    equal to single applies."""
    say("wide column batch")
    vg = _vg()
    torch = _torch()
    specs = [(3, 512, "helmholtz", 150.0), (3, 512, "laplace", 0.0), (3, 64, "helmholtz", 20.0)]
    plans = [vg.Plan(d, N, kind, k, precision="fp32") for d, N, kind, k in specs]
    rng = np.random.default_rng(512)
    fs = [torch.from_numpy((rng.standard_normal((N,) * d) + 1j * rng.standard_normal((N,) * d)).astype(np.complex64)).cuda()
          for d, N, _, _ in specs]
    ref = singles(plans, fs)
    out = vg.apply_batched(plans, fs)
    torch.cuda.synchronize()
    for i, (a, b) in enumerate(zip(out, ref)):
        assert torch.equal(a, b), i
    del plans, fs, ref, out
    torch.cuda.empty_cache()


def test_batched_fp64_matches_single_applies():
    say("fp64 batch")
    vg = _vg()
    torch = _torch()
    specs = [(3, 16, "helmholtz", 6.0), (3, 16, "laplace", 0.0), (3, 24, "helmholtz", 2.0), (2, 32, "laplace", 0.0)]
    plans = [vg.Plan(d, N, kind, k, precision="fp64") for d, N, kind, k in specs]
    fs = [dev(random_density(70 + i, d, N), "fp64") for i, (d, N, _, _) in enumerate(specs)]
    ref = singles(plans, fs)
    out = vg.apply_batched(plans, fs)
    torch.cuda.synchronize()
    for i, (a, b) in enumerate(zip(out, ref)):
        assert torch.equal(a, b), i


def test_batched_inside_caller_graph_capture():
    """After one eager call with the same arrays, a batched apply can be
    recorded into the caller's own graph; replays follow new density values."""
    say("caller capture")
    vg = _vg()
    torch = _torch()
    specs = [(3, 32, "helmholtz", 9.0), (3, 32, "helmholtz", 5.0), (3, 48, "laplace", 0.0)]
    plans = [vg.Plan(d, N, kind, k, precision="fp32") for d, N, kind, k in specs]
    fs = [dev(random_density(90 + i, d, N)) for i, (d, N, _, _) in enumerate(specs)]
    outs = [torch.empty_like(f) for f in fs]
    ws = torch.empty(vg.batched_workspace_size(plans), dtype=torch.uint8, device="cuda")
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        vg.apply_batched(plans, fs, outs, workspace=ws, stream=s)  # eager: builds the batch entry
    s.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        vg.apply_batched(plans, fs, outs, workspace=ws, stream=s)
    torch.cuda.synchronize()
    for r in range(3):
        for f in fs:
            f.mul_(complex(0.0, 1.0 + r))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        ref = singles(plans, fs)
        torch.cuda.synchronize()
        for i, (a, b) in enumerate(zip(outs, ref)):
            assert torch.equal(a, b), (r, i)


def test_batched_first_call_under_capture_is_refused():
    say("capture refusal")
    vg = _vg()
    torch = _torch()
    plans = [vg.Plan(3, 16, "laplace", precision="fp32")]
    fs = [dev(random_density(99, 3, 16))]
    outs = [torch.empty_like(fs[0])]
    ws = torch.empty(vg.batched_workspace_size(plans), dtype=torch.uint8, device="cuda")
    s = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    with pytest.raises(vg.VGError, match="NOT_CAPTURABLE|capture"):
        with torch.cuda.graph(g, stream=s):
            vg.apply_batched(plans, fs, outs, workspace=ws, stream=s)
    torch.cuda.synchronize()


@pytest.mark.parametrize("d,N,kernel,k,tune", [(3, 64, "helmholtz", 20.0, "quick"), (3, 48, "laplace", 0.0, "full"),
                                               (2, 2048, "laplace", 0.0, "quick"), (2, 128, "helmholtz", 30.0, "full")])
def test_autotuned_plans_agree_with_default_layout(d, N, kernel, k, tune, monkeypatch):
    """Plans built with the autotuner (timed layouts: pitch padding, tile
    order, four-step split, generic kernels) compute the same operator: equal
    to the default plan to FP32 rounding, bitwise when the default layout won."""
    say("autotune", d, N, kernel, k, tune)
    monkeypatch.setenv("VG_TUNE_CACHE", "")  # always time here: no persistent cache
    vg = _vg()
    torch = _torch()
    f = dev(random_density(120 + N, d, N))
    base = vg.Plan(d, N, kernel, k, precision="fp32")
    tuned = vg.Plan(d, N, kernel, k, precision="fp32", tune=tune)
    info = tuned.info
    say("  chosen", {key: info[key] for key in ("tune_ms", "tune_candidates", "pad_bytes", "xcd_map",
                                                  "four_step_L1", "generic_passes")})
    assert info["tune_candidates"] >= 4 and info["tune_ms"] > 0.0
    a = base.apply(f)
    b = tuned.apply(f)
    ga = base.gradient(f)[1]
    gb = tuned.gradient(f)[1]
    torch.cuda.synchronize()
    assert (torch.linalg.vector_norm(a - b) / torch.linalg.vector_norm(a)).item() <= 2e-6
    assert (torch.linalg.vector_norm(ga - gb) / torch.linalg.vector_norm(ga)).item() <= 2e-6
    if info["pad_bytes"] == 256 and info["xcd_map"] == 1 and info["four_step_L1"] == 0 and not info["generic_passes"]:
        assert torch.equal(a, b)


def test_batched_mixed_radix_lengths_equal_single_applies():
    """Batches over the mixed-radix lengths (2N = 100, 200, 300, 400): grouped
    launches where grouped kernels exist (300 launches per density), every
    output bitwise equal to the single apply."""
    say("mixed-radix batch")
    vg = _vg()
    torch = _torch()
    specs = [(3, 50, "helmholtz", 12.0), (3, 50, "laplace", 0.0), (3, 100, "helmholtz", 25.0),
             (3, 100, "helmholtz", 30.0), (3, 150, "laplace", 0.0), (2, 200, "helmholtz", 40.0),
             (2, 200, "laplace", 0.0), (2, 100, "helmholtz", 20.0)]
    plans = [vg.Plan(d, N, kind, k, precision="fp32") for d, N, kind, k in specs]
    fs = [dev(random_density(1500 + i, d, N)) for i, (d, N, _, _) in enumerate(specs)]
    ref = singles(plans, fs)
    out = vg.apply_batched(plans, fs)
    torch.cuda.synchronize()
    for i, (a, b) in enumerate(zip(out, ref)):
        assert torch.equal(a, b), i


def test_tune_cache_reuses_the_choice(tmp_path, monkeypatch):
    """The autotuner's persistent cache: the first tuned plan times its
    candidates and stores the choice; a second plan with the same key takes it
    without timing and computes bit for bit the same; a corrupt file or a
    stale entry (another library build) makes the next plan tune again."""
    import json
    vg = _vg()
    torch = _torch()
    path = tmp_path / "tune.json"
    monkeypatch.setenv("VG_TUNE_CACHE", str(path))
    fields = ("pad_bytes", "xcd_map", "four_step_L1", "generic_passes")
    f = dev(random_density(77, 3, 64))
    p1 = vg.Plan(3, 64, "helmholtz", 20.0, tune="quick")
    say("  first", p1.info["tune_cached"], p1.info["tune_candidates"], p1.info["tune_ms"])
    assert p1.info["tune_cached"] == 0 and p1.info["tune_candidates"] >= 4
    doc = json.loads(path.read_text())
    assert doc["format"] == "vgconv-tune-1" and len(doc["entries"]) == 1
    key = next(iter(doc["entries"]))
    assert "d=3;N=64;table=complex;precision=fp32;mode=quick" in key
    p2 = vg.Plan(3, 64, "helmholtz", 7.0, tune="quick")  # same key: k does not enter it
    say("  second", p2.info["tune_cached"], p2.info["tune_candidates"], p2.info["tune_ms"])
    assert p2.info["tune_cached"] == 1 and p2.info["tune_candidates"] == 0
    assert all(p2.info[x] == p1.info[x] for x in fields)
    p3 = vg.Plan(3, 64, "helmholtz", 20.0, tune="quick")
    a, b = p1.apply(f), p3.apply(f)
    torch.cuda.synchronize()
    assert p3.info["tune_cached"] == 1 and torch.equal(a, b)
    # corrupt file: tuned again, file rewritten
    path.write_text('{"format": "vgconv-tune-1", "entries": {')
    p4 = vg.Plan(3, 64, "helmholtz", 20.0, tune="quick")
    assert p4.info["tune_cached"] == 0 and p4.info["tune_candidates"] >= 4
    assert key in json.loads(path.read_text())["entries"]
    # stale entry: the same grid under another library build is not reused
    doc = json.loads(path.read_text())
    doc["entries"] = {key.rsplit("build=", 1)[0] + "build=0000000000000000": doc["entries"][key]}
    path.write_text(json.dumps(doc))
    p5 = vg.Plan(3, 64, "helmholtz", 20.0, tune="quick")
    assert p5.info["tune_cached"] == 0 and p5.info["tune_candidates"] >= 4
    # an unwritable location (below a regular file) is not an error
    (tmp_path / "afile").write_text("x")
    monkeypatch.setenv("VG_TUNE_CACHE", str(tmp_path / "afile" / "tune.json"))
    p6 = vg.Plan(3, 32, "laplace", 0.0, tune="quick")
    assert p6.info["tune_candidates"] >= 1
