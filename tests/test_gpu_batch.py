"""Batched uneven heat domains (by default one launch per k steps for all
domains, all launches in one graph launch; or one persistent kernel per run,
items of every domain, tile and group taken from a device queue;
autotuned tiles and temporal-blocking depth): every domain equals the
oracle's FP32 steps bit for bit (small domains, every depth, step counts that
are not multiples of the depth, odd and even numbers of groups), both modes
and the per-domain launch baseline agree bit for bit (the 64-domain workload
at full size), and a persistent launch whose bounded wait gives up ends
normally and is reported."""
import os

import numpy as np
import pytest
import torch

import oracle as O
from paper_2109_05410_amd import _lib as L
from paper_2109_05410_amd import api, inputs

pytestmark = pytest.mark.gpu
DEV = "cuda"


@pytest.mark.parametrize("steps", [7, 8, 1])
def test_small_uneven_domains_match_oracle(steps, tmp_path):
    shapes = [(9, 17, 33), (64, 64, 64), (100, 40, 70), (5, 3, 130), (1, 1, 1), (31, 129, 66)]
    u0 = [inputs.heat_uniform(s, seed=i) for i, s in enumerate(shapes)]
    fields = [torch.from_numpy(u).to(DEV) for u in u0]
    b = api.HeatBatch(fields, alpha=0.1, tune=True, tune_cache=str(tmp_path / "tune.json"))
    b.run(steps)
    torch.cuda.synchronize()
    for u, f in zip(u0, fields):
        assert np.array_equal(f.cpu().numpy(), O.heat7_f32(u, 0.1, steps))
    assert os.path.exists(tmp_path / "tune.json")
    # the per-domain baseline computes the same
    fields2 = [torch.from_numpy(u).to(DEV) for u in u0]
    b2 = api.HeatBatch(fields2, alpha=0.1, tune=False, tune_cache=str(tmp_path / "tune.json"))
    b2.run_per_domain(steps)
    torch.cuda.synchronize()
    for f, g in zip(fields, fields2):
        assert torch.equal(f, g)


@pytest.mark.parametrize("depth,steps", [(2, 7), (2, 8), (4, 9), (4, 3), (1, 5)])
def test_forced_depth_matches_oracle(depth, steps):
    """Temporal blocking: k steps per launch over tiles with a k-cell halo
    give the single-step result bit for bit, on domains smaller than a tile
    and domains spanning several tiles and z chunks."""
    shapes = [(9, 17, 33), (140, 40, 70), (5, 3, 130), (1, 1, 1), (31, 129, 66), (3, 2, 1)]
    u0 = [inputs.heat_uniform(s, seed=20 + i) for i, s in enumerate(shapes)]
    fields = [torch.from_numpy(u).to(DEV) for u in u0]
    b = api.HeatBatch(fields, alpha=0.1, tune=False, depth=depth)
    assert b.depth == depth
    b.run(steps)
    torch.cuda.synchronize()
    for u, f in zip(u0, fields):
        assert np.array_equal(f.cpu().numpy(), O.heat7_f32(u, 0.1, steps))
    fields2 = [torch.from_numpy(u).to(DEV) for u in u0]
    b2 = api.HeatBatch(fields2, alpha=0.1, tune=False, depth=depth)
    b2.run_per_domain(steps)
    torch.cuda.synchronize()
    for f, g in zip(fields, fields2):
        assert torch.equal(f, g)


def test_graph_replays():
    shapes = [(16, 16, 16), (20, 24, 28)]
    u0 = [inputs.heat_uniform(s, seed=10 + i) for i, s in enumerate(shapes)]
    fields = [torch.from_numpy(u).to(DEV) for u in u0]
    b = api.HeatBatch(fields, tune=False)
    for _ in range(3):
        b.run(4)
    torch.cuda.synchronize()
    for u, f in zip(u0, fields):
        assert np.array_equal(f.cpu().numpy(), O.heat7_f32(u, 0.1, 12))


def test_full_size_batched_workload(tmp_path):
    """64 cubes with sides uniform in [64, 384], 200 steps: batched graph
    launch equals per-domain launches bit for bit; the smallest domain
    equals the oracle."""
    sides = inputs.batch_sides()
    fields = [torch.from_numpy(inputs.heat_uniform((s, s, s), seed=3 + j)).to(DEV) for j, s in enumerate(sides)]
    ref = [f.clone() for f in fields]
    ref2 = [f.clone() for f in fields]
    b = api.HeatBatch(fields, tune=True, tune_cache=str(tmp_path / "tune.json"))
    b.run(200, check=True)
    b2 = api.HeatBatch(ref, tune=False, tune_cache=str(tmp_path / "tune.json"))
    b2.run_per_domain(200)
    b3 = api.HeatBatch(ref2, tune=False, tune_cache=str(tmp_path / "tune.json"))
    b3.set_persistent(True)
    b3.run(200, check=True)
    torch.cuda.synchronize()
    for f, g, h in zip(fields, ref, ref2):
        assert torch.equal(f, g)
        assert torch.equal(f, h)
    j = int(np.argmin(sides))
    s = int(sides[j])
    want = O.heat7_f32(inputs.heat_uniform((s, s, s), seed=3 + j), 0.1, 200)
    assert np.array_equal(fields[j].cpu().numpy(), want)


def test_tuning_leaves_the_states_unchanged(tmp_path):
    """Creating a batch with tuning times tile candidates on single domains
    and one launch per depth over the whole batch; those launches write only
    the scratch buffers, so every domain's state is what the caller put in,
    and a run afterwards equals the oracle."""
    shapes = [(40, 36, 64), (17, 9, 33), (64, 64, 64), (1, 1, 1), (30, 70, 20)]
    u0 = [inputs.heat_uniform(s, seed=20 + i) for i, s in enumerate(shapes)]
    fields = [torch.from_numpy(u).to(DEV) for u in u0]
    b = api.HeatBatch(fields, alpha=0.1, tune=True, tune_cache=str(tmp_path / "tune.json"))
    torch.cuda.synchronize()
    assert b.depth in (1, 2, 4)
    for u, f in zip(u0, fields):
        assert np.array_equal(f.cpu().numpy(), u)
    b.run(6)
    torch.cuda.synchronize()
    for u, f in zip(u0, fields):
        assert np.array_equal(f.cpu().numpy(), O.heat7_f32(u, 0.1, 6))


@pytest.mark.parametrize("persistent", [True, False])
@pytest.mark.parametrize("depth,steps", [(4, 8), (4, 12), (4, 6), (2, 5), (1, 3), (1, 4)])
def test_persistent_and_launch_modes_match_oracle(depth, steps, persistent):
    """Both modes, with groups only at the batch depth (even and odd counts)
    and with depth-1 groups after them."""
    shapes = [(40, 36, 64), (17, 9, 33), (64, 64, 64), (1, 1, 1), (130, 70, 20), (8, 300, 12)]
    u0 = [inputs.heat_uniform(s, seed=40 + i) for i, s in enumerate(shapes)]
    fields = [torch.from_numpy(u).to(DEV) for u in u0]
    b = api.HeatBatch(fields, alpha=0.1, tune=False, depth=depth)
    b.set_persistent(persistent)
    b.run(steps, check=True)
    for u, f in zip(u0, fields):
        assert np.array_equal(f.cpu().numpy(), O.heat7_f32(u, 0.1, steps))
    # a second run on the same graph continues from the state
    b.run(steps, check=True)
    for u, f in zip(u0, fields):
        assert np.array_equal(f.cpu().numpy(), O.heat7_f32(u, 0.1, 2 * steps))


@pytest.mark.parametrize("cfg", [9, 10, 11])
def test_every_depth4_tile_matches_oracle(cfg, tmp_path):
    """The three 4-step tile shapes the autotuner chooses from (z chunks of
    64, 32 and 128 planes), forced through the tuning cache."""
    shapes = [(140, 40, 70), (9, 17, 33), (200, 31, 66)]
    u0 = [inputs.heat_uniform(s, seed=60 + i) for i, s in enumerate(shapes)]
    fields = [torch.from_numpy(u).to(DEV) for u in u0]
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    cache = tmp_path / "tune.json"
    cache.write_text("{" + ",".join(f'"{arch}/heat7/bucket{b}/k4": {cfg}' for b in range(9)) + "}")
    b = api.HeatBatch(fields, alpha=0.1, tune=False, tune_cache=str(cache), depth=4)
    tiles = {b.tile(i) for i in range(len(shapes))}
    assert tiles == {(64, 16, {9: 64, 10: 32, 11: 128}[cfg], 4)}
    b.run(9, check=True)
    for u, f in zip(u0, fields):
        assert np.array_equal(f.cpu().numpy(), O.heat7_f32(u, 0.1, 9))


def test_persistent_wait_gives_up_and_is_reported():
    """A wait that is never satisfied (test hook) gives up after its poll
    limit; every workgroup leaves, the kernel ends, check() reports it, and
    the next run (default limit) is correct again."""
    shapes = [(40, 36, 64), (64, 64, 64)]
    u0 = [inputs.heat_uniform(s, seed=80 + i) for i, s in enumerate(shapes)]
    fields = [torch.from_numpy(u).to(DEV) for u in u0]
    b = api.HeatBatch(fields, alpha=0.1, tune=False, depth=4)
    b.set_persistent(True)
    b.set_wait_limit(1000, never_satisfied=True)
    b.run(8)
    with pytest.raises(L.OocsError) as e:
        b.check()
    assert e.value.code == L.OOCS_E_TIMEOUT
    b.check()  # the status was cleared
    b.set_wait_limit(1 << 21)
    for u, f in zip(u0, fields):
        f.copy_(torch.from_numpy(u))
    b.run(8, check=True)
    for u, f in zip(u0, fields):
        assert np.array_equal(f.cpu().numpy(), O.heat7_f32(u, 0.1, 8))
