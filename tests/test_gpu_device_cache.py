"""The library's device-buffer cache: handles set up after others were
released reuse their buffers, which hold the old contents, so every result
must be the same bit for bit as from fresh memory; the oracle judges one of
them to the interior-solve tolerance (1e-9 relative, element by element per
block: FP64 GEMV form of the same LU factors, cond(A_jj) < 1e5)."""
import numpy as np
import pytest

from tests.gpu_systems import blocks_of, blockwise_err, gpu_precond, make_system, oracle_precond

torch = pytest.importorskip("torch")
from paper_1104_3349_amd import addns  # noqa: E402

pytestmark = pytest.mark.gpu


def _apply(S, pc):
    y = torch.from_numpy(np.random.default_rng(7).standard_normal(S.N)).cuda()
    x = torch.empty_like(y)
    addns.apply_precond(pc, y, x)
    torch.cuda.synchronize()
    return y.cpu().numpy(), x.cpu().numpy()


def test_reused_buffers_give_identical_results():
    A = make_system(n=24, nu=0.05, m=4, sz=16, seed=9)
    B = make_system(n=40, nu=0.02, m=8, sz=16, seed=3)
    part_a, pc = gpu_precond(A)
    y, first = _apply(A, pc)
    del pc
    # a larger and a smaller system on buffers the first one released
    for S in (B, A, B):
        if S is A:
            part, pc = gpu_precond(A, part=part_a)
        else:
            part, pc = gpu_precond(S, coarse=8)
        _, x = _apply(S, pc)
        if S is A:
            assert np.array_equal(x, first)
        del pc
    freed = addns.release_cached_memory()
    assert freed > 0
    assert addns.release_cached_memory() == 0
    part, pc = gpu_precond(A, part=part_a)
    _, x = _apply(A, pc)
    assert np.array_equal(x, first)
    ora = oracle_precond(A)
    err = blockwise_err(x, ora.apply(y), blocks_of(ora.part))
    assert err <= 1e-9, err
