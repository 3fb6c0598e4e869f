"""The allocation-free learned-correction call (fsi_mlp_forward_noalloc)
against the allocating one (fsi_mlp_forward), through the C ABI.

The allocation-free call stages the FP32 residual and correction in the
library's per-GPU array instead of buffers allocated per call; both run the
same kernels on the same values, so the results are identical (bit-exact).
Two calls in a row share the array: the second, on a smaller level, must not
see the first one's contents."""
import numpy as np
import pytest

from conftest import system

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def _weights(k_in, d, seed):
    rng = np.random.default_rng(seed)
    return [(rng.standard_normal((k_in, 64)) * np.sqrt(2.0 / k_in)).astype(np.float32),
            (rng.standard_normal((64, 64)) * np.sqrt(2.0 / 64)).astype(np.float32),
            (rng.standard_normal((64, d)) * np.sqrt(1.0 / 64)).astype(np.float32)]


def _solver(name, precision):
    from paper_1801_05648_amd import FsiSolver
    sysm = system(name)
    s = FsiSolver.from_system(sysm, device=0)
    s.build_precond(precision, max_coarse=40)  # two or more levels: the learned smoother needs them
    d = sysm.dim
    for which in ("H_M", "H_SIG"):
        s.mlp_set_weights(which, *_weights(3 ** d * d, d, seed=5))
    return s


@pytest.mark.parametrize("precision", ["f32", "f64"])
def test_noalloc_forward_matches_the_allocating_call(precision):
    # first call on the larger 2D system, second on the smaller one
    for name, which in (("c2", "H_M"), ("c1", "H_SIG"), ("c1", "H_M")):
        s = _solver(name, precision)
        from paper_1801_05648_amd import fsi
        n = s._hier_len(fsi.HIERARCHIES[which])
        b = torch.from_numpy(np.random.default_rng(n).standard_normal(n)).to("cuda:0")
        ref = s.mlp_forward(which, b)
        x = torch.full_like(b, float("nan"))
        s.mlp_forward_noalloc(which, b, x)
        torch.cuda.synchronize()
        print(f"{name} {which} {precision}: n={n}, max |diff| {float((x - ref).abs().max()):.3e}")
        assert torch.isfinite(ref).all()
        assert torch.equal(x, ref), (name, which)
        s.close()
