"""smc_kernel_resample_noalloc (scratch in a static device array, no allocation) gives the
ancestors of smc_kernel_resample bit for bit, on consecutive calls whose sizes shrink (the
static scratch keeps the previous call's contents), up to its size limit; a size beyond
the limit is refused before any device work."""
import numpy as np
import pytest

from gpu_util import dev, say, torch_cuda
from paper_2604_03271_amd import native

pytestmark = pytest.mark.gpu


def _weights(rng, P, kind):
    if kind == "dir":
        return rng.dirichlet(np.full(P, 0.7))
    w = np.exp(-rng.exponential(30.0, P))
    return w / w.sum()


def test_noalloc_resample_equals_allocating_entry_point():
    torch = torch_cuda()
    rng = np.random.default_rng(77)
    limit = 1 << 20   # SMC_NOALLOC_MAX_P
    for P, M, kind in ((65536, 4096, "dir"), (1000, 250, "spiky"), (limit, limit // 16, "dir"), (7, 7, "dir")):
        W_ = _weights(rng, P, kind)
        r = int(rng.integers(0, 2 ** 32))
        say("noalloc resample", P, M, kind, r)
        w_dev = dev(W_, torch.float64)
        a_ref = torch.zeros(M, dtype=torch.int32, device="cuda")
        native.smc_kernel_resample(w_dev, M, r, a_ref)
        a = torch.full((M,), -1, dtype=torch.int32, device="cuda")
        native.smc_kernel_resample_noalloc(w_dev, M, r, a)
        torch.cuda.synchronize()
        assert np.array_equal(a.cpu().numpy(), a_ref.cpu().numpy()), (P, M)


def test_noalloc_resample_refuses_beyond_limit():
    torch = torch_cuda()
    P = (1 << 20) + 1
    w = torch.full((P,), 1.0 / P, dtype=torch.float64, device="cuda")
    a = torch.zeros(16, dtype=torch.int32, device="cuda")
    with pytest.raises(native.SMCError) as e:
        native.smc_kernel_resample_noalloc(w, 16, 0, a)
    assert e.value.status == native.SMC_EINVAL
