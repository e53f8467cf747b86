"""The autotuner on the GPU: it picks a shape, installs it, and the library
stays correct with it."""
import numpy as np
import pytest
import torch

import oracle

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("mode,dim,n", [("f32", 3, 16), ("f32", 2, 10), ("bf16x3", 3, 6)])
def test_autotune_installs_a_correct_shape(mode, dim, n):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1304_7054_amd as kron
    from paper_1304_7054_amd import tune
    code = tune.MODES[mode]
    try:
        r = tune.tune_case(mode, dim, n, target_bytes=16 << 20, reps=3)
        assert kron.kron_get_launch(code, dim, n) == (r["blocks_per_cu"], r["variant"])
        assert r["ms"] > 0
        rng = np.random.default_rng(5)
        batch = 300
        mats = [rng.uniform(-1, 1, n * n).astype(np.float32) for _ in range(dim)]
        X = rng.standard_normal(batch * n ** dim).astype(np.float32)
        tm = [torch.from_numpy(m).cuda() for m in mats]
        tx = torch.from_numpy(X).cuda()
        ty = torch.full_like(tx, float("nan"))
        fn = {("f32", 2): kron.kron2d_batched_f32, ("f32", 3): kron.kron3d_batched_f32,
              ("bf16x3", 3): kron.kron3d_batched_f32_bf16x3}[(mode, dim)]
        fn(n, *tm, tx, ty, batch)
        torch.cuda.synchronize()
        want = (oracle.kron2d if dim == 2 else oracle.kron3d)(n, *mats, X, batch, "f64")
        got = ty.cpu().numpy()
        assert np.linalg.norm(got - want) <= 1e-5 * np.linalg.norm(want)
    finally:
        kron.kron_set_launch(code, dim, n, -1, 0)
