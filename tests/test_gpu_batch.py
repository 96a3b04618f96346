"""The K-field batch (K fields sharing one weight set) against the FP64 oracle,
at every slice width of the LDS-staged kernels.

Each field is its own Gaussian pulse on the PEC square; the batch advances
them together for 300 steps.  The 16-field slices (the width the tuner picks
on the 250k-node benchmark set), 8- and 4-field slices compute every field
with the same arithmetic in the same order, one item per workgroup or in the
persistent kernels with staging wavefronts, so they agree bit for bit, and
the global-gather kernels to rounding; each field matches the oracle's single
FP64 run of that pulse within the FP32 bar.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2508_18205_amd import Solver  # noqa: E402
from oracle import setup as osetup, step as ostep  # noqa: E402
from synth import configs  # noqa: E402


def _announce(msg):
    print(msg, flush=True)


@pytest.mark.parametrize("K", [16, 64])
def test_batch_slice_widths_per_field_vs_oracle(K):
    w = configs.batched_2d(n_side=40, K=K, chat=1e-3, steps=300)
    _announce(f"batch K={K}: N={w.N}, {w.steps} steps")
    s = Solver.from_workload(w, precision="f32", K=K)
    H0 = np.zeros((K, w.N, 2))
    outs = []
    runs = ((16, 1), (8, 1), (4, 1), (16, 2), (8, 2), (4, 2), (8, 0))
    for persist, lds in runs:
        s.set_variant(block=256, xcd=1, lds=lds, persist=persist)
        st = s.state_batched(w.E0_batch, H0)
        s.run(st, w.steps, use_graph=True)
        outs.append((s.to_original(st.E)[:, 0, :], s.to_original(st.H)))
    for o in outs[1:6]:
        assert np.array_equal(o[0], outs[0][0]) and np.array_equal(o[1], outs[0][1])
    g = outs[6]
    assert np.abs(g[0] - outs[0][0]).max() <= 1e-6 * np.abs(outs[0][0]).max()
    assert np.abs(g[1] - outs[0][1]).max() <= 1e-6 * np.abs(outs[0][1]).max()
    Eb, Hb = outs[0]
    oh, oe = osetup.operators(w)
    gamma = ostep.hv_gamma(w.hv_c, w.alpha, w.h)
    keep = ostep.pec_keep(w.flags, 2)
    worst = 0.0
    for k in (range(K) if K <= 16 else range(0, K, 7)):
        Eo, Ho, _, _ = ostep.run(w.E0_batch[k], np.zeros((w.N, 2)), oh, oe, w.dt, w.steps, gamma, w.dt, keep)
        e = max(np.abs(Eb[:, k] - Eo[:, 0]).max() / np.abs(Eo).max(), np.abs(Hb[:, :, k] - Ho).max() / np.abs(Ho).max())
        worst = max(worst, e)
    _announce(f"  slice widths 16/8/4, per item and persistent, identical; worst field vs oracle {worst:.2e}")
    assert worst < 1e-5
