"""The model matrix fills of Sec. IV.A on the GPU (eqs.(Atrig), (Agau),
(Acond)) against the oracle: dense FP64 within 1e-13 relative, FP32 within
2e-5; the filtered dense fill equal to the dense one where u <= alpha and
zero elsewhere; the pre-selected fill's indices bit-exact and its values
equal to the dense ones; a capacity below the count is refused."""
import sys

import numpy as np
import pytest

import oracle.model as MD
from inputs import SEED

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    import paper_1508_07441_amd as P
    c = P.Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("kind,K,M", [(0, 7, 96), (1, 5, 70), (0, 1, 257)])
def test_model_fill_parity(ctx, kind, K, M):
    import paper_1508_07441_amd as P
    name = "trig" if kind == 0 else "gauss"
    ref = MD.model_fill(name, M, K, SEED)
    say(f"[model {name} K={K} M={M}] dense FP64")
    A, _ = ctx.model_fill(kind, 0, M, K, seed=SEED)
    assert np.all(np.abs(A - ref) <= 1e-13 * np.maximum(np.abs(ref), 1.0))
    say(f"[model {name}] dense FP32")
    A32, _ = ctx.model_fill(kind, 0, M, K, seed=SEED, precision=P.WPCD_MIXED)
    assert np.all(np.abs(A32 - ref) <= 2e-5 * np.maximum(np.abs(ref), 1.0))
    alpha = 0.05
    idx_o, val_o = MD.model_fill(name, M, K, SEED, alpha)
    say(f"[model {name}] filtered")
    F, _ = ctx.model_fill(kind, 1, M, K, alpha=alpha, seed=SEED)
    keep = np.zeros(M * M, bool)
    keep[idx_o] = True
    assert np.array_equal(F.ravel()[keep], A.ravel()[keep])
    assert np.all(F.ravel()[~keep] == 0.0)
    say(f"[model {name}] selected")
    (idx, val), _ = ctx.model_fill(kind, 2, M, K, alpha=alpha, seed=SEED)
    assert np.array_equal(idx, idx_o)
    assert np.array_equal(val, A.ravel()[idx])
    with pytest.raises(P.WpcdError) as ei:
        ctx.model_fill(kind, 2, M, K, alpha=alpha, seed=SEED, cap=max(idx_o.size - 1, 0))
    assert ei.value.status == P.WPCD_E_INVALID
