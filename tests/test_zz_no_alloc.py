"""The allocation-free apply (addns_apply_precond_static) against the
ordinary apply (addns_apply_precond): the same kernels on the same factors,
so the outputs agree bit for bit.  Two calls in a row share the static
array, the second on a smaller system; each must be exact, and the first
system's apply must still be exact after the second ran."""
import numpy as np
import pytest

from tests.gpu_systems import gpu_precond, make_system

torch = pytest.importorskip("torch")
from paper_1104_3349_amd import addns  # noqa: E402

pytestmark = pytest.mark.gpu


def _cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _both(pc, N, seed):
    y = _cuda(np.random.default_rng(seed).standard_normal(N))
    ref = torch.zeros(N, dtype=torch.float64, device="cuda")
    got = torch.full((N,), np.nan, dtype=torch.float64, device="cuda")
    addns.apply_precond(pc, y, ref)
    addns.apply_precond_static(pc, y, got)
    torch.cuda.synchronize()
    return got.cpu().numpy(), ref.cpu().numpy()


@pytest.mark.parametrize("kw", [dict(), dict(iprec=addns.F32, sprec=addns.F32, coarse=16)])
def test_static_apply_equals_apply_on_two_calls(kw):
    big = make_system(n=48, nu=0.005, m=6, sz=40, stretch=1.05, seed=7)
    small = make_system(n=16, nu=0.1, m=4, sz=64, seed=1001)
    _, pc_big = gpu_precond(big, **kw)
    _, pc_small = gpu_precond(small, **kw)
    for pc, S, seed in ((pc_big, big, 1), (pc_small, small, 2), (pc_big, big, 3)):
        got, ref = _both(pc, S.N, seed)
        assert np.isfinite(got).all()
        assert np.array_equal(got, ref)


def test_static_apply_argument_errors():
    S = make_system(n=12, nu=0.1, m=3, sz=16, seed=2)
    _, pc = gpu_precond(S)
    d = torch.zeros(S.N, dtype=torch.float64, device="cuda")
    with pytest.raises(addns.AddnsError) as e:
        addns.apply_precond_static(pc, d, d)
    assert e.value.code == addns.ERR_ARG
