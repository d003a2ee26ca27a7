"""The allocation-free weight gradient (epidmc_dn_wgrad_noalloc) against the entry point that
takes caller scratch (epidmc_dn_wgrad), through the C ABI: the same kernels in the same
chunk plan, so the two give the same bits.  Two calls in a row, the second on a smaller
shape, show that the library-held scratch keeps no state that a later call depends on; a
shape whose partial sums exceed the held scratch is refused before any launch."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

CASES = [  # (n, h, w, c_in, ld_in, c_out, k, with_bias): the first needs 7.4 M of the 10.5 M floats
    (2, 64, 96, 128, 128, 128, 3, True),
    (1, 33, 40, 64, 128, 64, 3, True),     # smaller, ragged, a channel slice of a wider input
    (3, 20, 30, 256, 256, 128, 1, False),  # 1x1, no bias gradient
]


@pytest.fixture(scope="module")
def D():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2510_24154_amd import denoise
    return denoise


def operands(case, seed):
    import torch
    n, h, w, ci, ldi, co, k, _ = case
    rng = np.random.default_rng(seed)
    x = torch.as_tensor(rng.standard_normal((n, h, w, ldi)).astype(np.float32)).to(torch.bfloat16).cuda()
    g = torch.as_tensor(rng.standard_normal((n, h, w, co)).astype(np.float32)).to(torch.bfloat16).cuda()
    return x[..., :ci], g


def test_noalloc_wgrad_matches_the_scratch_entry_point(D):
    import torch
    for i, case in enumerate(CASES):
        k, with_bias = case[6], case[7]
        print("no-alloc wgrad case", case, flush=True)
        x, g = operands(case, 100 + i)
        dw_ref, db_ref = D.wgrad(x, g, k, with_bias=with_bias)
        dw, db = D.wgrad_noalloc(x, g, k, with_bias=with_bias)
        torch.cuda.synchronize()
        assert torch.isfinite(dw_ref).all() and float(dw_ref.abs().sum()) > 0
        assert torch.equal(dw, dw_ref), case
        if with_bias:
            assert torch.equal(db, db_ref), case
        else:
            assert db is None


def test_noalloc_wgrad_refuses_shapes_beyond_its_scratch(D):
    """c_in = c_out = 512, 3x3, 2048 pixels: the chunk plan needs 11.8 M floats of partial
    sums, more than the 10.5 M the library holds (checked on the host before any launch)."""
    import torch
    from paper_2510_24154_amd import EpidmcError
    x = torch.zeros((1, 32, 64, 512), dtype=torch.bfloat16, device="cuda")
    g = torch.zeros((1, 32, 64, 512), dtype=torch.bfloat16, device="cuda")
    with pytest.raises(EpidmcError) as e:
        D.wgrad_noalloc(x, g, 3)
    assert e.value.code == -5   # EPIDMC_E_WORKSPACE
