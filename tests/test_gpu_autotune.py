"""Plan options and the autotuner of the batched form: every option set (bottom-kernel threshold
and workgroup size, smoother tile width, fused or separate finest-level launches between
cycles, residual inside the Jacobian launch or separate) gives the same result bit for bit (the kernels do the same arithmetic in the same
order), and the autotuner restores the states it trials on and keeps the fastest set."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from swe_workloads import config1, config2, config4_instance  # noqa: E402

DEV = "cuda:0"


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _probs():
    return [config2(0, "sub"), config4_instance(7), config1(2), config4_instance(11)]


@pytest.mark.parametrize("prec_name", ["fp64", "fp32mg"])
def test_every_option_set_gives_the_same_solution(prec_name):
    from paper_2505_10857_amd import NMG_FP32_MG, NMG_FP64, BatchSolver1D
    prec = NMG_FP64 if prec_name == "fp64" else NMG_FP32_MG
    probs = _probs()
    ref = None
    for c in range(32):
        cells, split, tile, sres = BatchSolver1D.tune_candidate(c)
        s = BatchSolver1D(probs, device=DEV, precision=prec)
        s.set_options(cells, smooth_tile=tile, split_finest=split, split_residual=sres)
        opt = s.options()
        assert (opt["bottom_cells"], opt["split_finest"], opt["smooth_tile"], opt["split_residual"]) == \
            (cells, split, tile, sres)
        assert opt["fused_finest"] == (split == 0)
        Us = s.states()
        st = s.solve(Us, use_graph=True)
        out = [u.cpu().numpy() for u in Us]
        print(prec_name, cells, split, tile, sres, [x[0] for x in st])
        assert all(x[1] == 0 for x in st)
        if ref is None:
            ref = (out, st)
        else:
            for a, b in zip(out, ref[0]):
                assert np.array_equal(a, b)
            assert [x[0] for x in st] == [x[0] for x in ref[1]]


def test_autotune_restores_states_and_keeps_a_valid_option():
    from paper_2505_10857_amd import NMG_FP64, BatchSolver1D
    probs = _probs()
    s = BatchSolver1D(probs, device=DEV, precision=NMG_FP64)
    Us = s.states()
    before = [u.clone() for u in Us]
    best, times = s.autotune(Us, trial_steps=2)
    print("autotune", best, times)
    assert best["bottom_cells"] in (256, 512, 1024, 2048)
    assert best["smooth_tile"] in (256, 512) and best["split_finest"] in (0, 1)
    assert len(times) == 32 and all(t > 0 for t in times.values())
    key = (best["bottom_cells"], best["split_finest"], best["smooth_tile"], best["split_residual"])
    assert key == min(times, key=times.get)
    opt = s.options()
    assert (opt["bottom_cells"], opt["split_finest"], opt["smooth_tile"], opt["split_residual"]) == key
    for a, b in zip(Us, before):
        assert torch.equal(a, b)
    st = s.solve(Us, use_graph=True)
    assert all(x[1] == 0 for x in st)


def test_bad_option_is_rejected():
    from paper_2505_10857_amd import BatchSolver1D, NmgError
    s = BatchSolver1D([config1(0)], device=DEV)
    s.set_options(1024, smooth_tile=512)
    for bad in (dict(bottom_cells=300), dict(bottom_cells=512, smooth_tile=300),
                dict(bottom_cells=512, split_finest=2), dict(bottom_cells=512, split_residual=3)):
        with pytest.raises(NmgError):
            s.set_options(**bad)
        opt = s.options()   # a rejected set leaves the plan as it was
        assert (opt["bottom_cells"], opt["smooth_tile"], opt["split_finest"]) == (1024, 512, 0)
