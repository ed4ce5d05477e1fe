"""The allocation-free dense run (vpmc_run_spots_noalloc, static device
scratch) against vpmc_run_spots on the same arguments: the same bits of
dose, standard error and ledger, on consecutive calls of shrinking size (the
scratch keeps the previous call's contents), and a clear error for a run
that does not fit in the scratch."""
import sys

import numpy as np
import pytest

from paper_2307_01416_amd import inputs as I

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def eng():
    import torch
    assert torch.cuda.is_available()
    from paper_2307_01416_amd import vpmc as V
    e = V.Engine(0)
    yield e
    e.close()


def _run_noalloc(eng, case, scen, n_batches, seed):
    import torch
    from paper_2307_01416_amd import vpmc as V
    nx, ny, nz = case.geometry.shape
    dev = torch.device("cuda", 0)
    dose = torch.full((len(scen), nz, ny, nx), -1.0, dtype=torch.float32, device=dev)
    sig = torch.full_like(dose, -1.0) if n_batches >= 2 else None
    led = np.zeros((len(scen), V.NLEDGER), np.float64)
    spots = case.fields[0].spots
    opts = V.make_opts(seed=seed, physics=case.physics, n_batches=n_batches, flags=V.DEVICE_PTRS,
                       stream=eng.stream_ptr())
    V.vpmc_run_spots_noalloc(eng.ctx, 0, V.spot_array(spots), len(spots), V.scenario_array(scen), len(scen),
                             opts, dose, sig, led)
    torch.cuda.synchronize()
    return dose, sig, led


def _compare(eng, case, scen, n_batches, seed=0):
    import torch
    eng.load_case(case)
    d0, s0, l0 = eng.run_dose(case, 0, scenarios=scen, n_batches=n_batches, sigma=n_batches >= 2, seed=seed)
    torch.cuda.synchronize()
    d1, s1, l1 = _run_noalloc(eng, case, scen, n_batches, seed)
    assert float(d0.max()) > 0.0
    assert torch.equal(d0, d1), float((d0 - d1).abs().max())
    if n_batches >= 2:
        assert torch.equal(s0, s1)
    assert np.array_equal(l0, l1)


def test_noalloc_equals_run_spots_on_shrinking_calls(eng):
    # first call: 64x64x200 water behind a 20 mm opening with range shifter,
    # two scenarios, 16 batches (19.7 MB of the scratch)
    big = I.config2(20.0, True, histories_per_case=200_000, shape=(64, 64, 200), seed=0)
    scen = [I.Scenario(), I.Scenario(shift_mm=(1.5, 0.0, 0.0), range_scale=1.035)]
    say("case noalloc config2-small 2 scenarios 16 batches")
    _compare(eng, big, scen, 16)
    # second call, smaller: config 1 (50x50x100), one scenario, 16 batches
    small = I.config1(n_histories=50_000, seed=3)
    say("case noalloc config1 16 batches")
    _compare(eng, small, small.scenarios, 16, seed=3)
    # third call, smaller still: straight mode without batches
    tiny = I.config1(n_histories=20_000, physics=0)
    say("case noalloc config1 straight no batches")
    _compare(eng, tiny, tiny.scenarios, 0)


def test_noalloc_rejects_runs_beyond_the_scratch(eng):
    from paper_2307_01416_amd import vpmc as V
    import torch
    c = I.config2(10.0, False, histories_per_case=1000, shape=(128, 128, 100))   # 1.64e6 voxels
    eng.load_case(c)
    say("case noalloc oversize")
    nx, ny, nz = c.geometry.shape
    dose = torch.full((1, nz, ny, nx), -1.0, dtype=torch.float32, device="cuda")
    sig = torch.full_like(dose, -1.0)
    spots = c.fields[0].spots
    opts = V.make_opts(physics=c.physics, n_batches=16, flags=V.DEVICE_PTRS, stream=eng.stream_ptr())
    with pytest.raises(V.VpmcError) as ei:
        V.vpmc_run_spots_noalloc(eng.ctx, 0, V.spot_array(spots), len(spots), V.scenario_array(c.scenarios), 1,
                                 opts, dose, sig, None)
    assert ei.value.code == V.E_OOM and "scratch" in str(ei.value)
    assert bool((dose == -1.0).all()) and bool((sig == -1.0).all())
    # the same grid fits without batches (8 B per voxel)
    opts = V.make_opts(physics=c.physics, n_batches=0, flags=V.DEVICE_PTRS, stream=eng.stream_ptr())
    V.vpmc_run_spots_noalloc(eng.ctx, 0, V.spot_array(spots), len(spots), V.scenario_array(c.scenarios), 1,
                             opts, dose, None, None)
    torch.cuda.synchronize()
    assert float(dose.max()) > 0.0
