"""kg_mlp_forward_noalloc (surrogate inference for callers that cannot
allocate device memory) against kg_mlp_forward on the same parameters and
inputs, through the C-ABI.  Both run the same kernels in the same order, so
the outputs must agree bit for bit.  Two calls in a row share the library's
scratch array, the second with fewer rows; the first spans more than one
scratch chunk (4032 rows at hidden = 128) and ends ragged."""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu

HIDDEN = 128


def test_no_alloc_forward_matches_forward(kg):
    rng = np.random.default_rng(7)
    params = rng.uniform(-0.3, 0.3, kg.kg_mlp_num_params(HIDDEN)).astype(np.float32)
    mean = np.array([2.2, 1.2, 1.3, 1.25], np.float32)
    stdev = np.array([1.0, 0.43, 0.41, 0.44], np.float32)
    stream = torch.cuda.current_stream()
    m = kg.kg_mlp_create(HIDDEN, 512, params, stream.cuda_stream)
    try:
        kg.kg_mlp_set_norm(m, mean, stdev)
        p_dev = torch.from_numpy(kg.kg_mlp_get_params(m, HIDDEN)).cuda()
        for n in (5000, 37):
            x = torch.from_numpy(np.stack([rng.uniform(0.5, 4.0, n)] +
                                          [rng.uniform(0.5, 2.0, n) for _ in range(3)],
                                          1).astype(np.float32)).cuda()
            ref = torch.empty((n, 2), dtype=torch.float32, device="cuda")
            got = torch.full((n, 2), float("nan"), dtype=torch.float32, device="cuda")
            kg.kg_mlp_forward(m, x, ref)
            before = torch.cuda.memory_allocated()
            kg.kg_mlp_forward_noalloc(HIDDEN, p_dev, x, got, mean, stdev, stream.cuda_stream)
            torch.cuda.synchronize()
            assert torch.cuda.memory_allocated() == before
            assert torch.isfinite(ref).all()
            assert torch.equal(got, ref), (n, (got - ref).abs().max().item())
    finally:
        torch.cuda.synchronize()
        kg.kg_mlp_destroy(m)


def test_no_alloc_forward_rejects_bad_arguments(kg):
    x = torch.zeros((4, 4), dtype=torch.float32, device="cuda")
    out = torch.zeros((4, 2), dtype=torch.float32, device="cuda")
    p = torch.zeros(kg.kg_mlp_num_params(8), dtype=torch.float32, device="cuda")
    with pytest.raises(kg.KGError) as e:
        kg.kg_mlp_forward_noalloc(1025, p, x, out)
    assert e.value.status == kg.KG_E_INVALID
    with pytest.raises(kg.KGError) as e:
        kg.kg_mlp_forward_noalloc(8, p, x, out, stdev=np.zeros(4, np.float32))
    assert e.value.status == kg.KG_E_INVALID
    # zero rows: a no-op
    kg.kg_mlp_forward_noalloc(8, p, x[:0], out[:0])
