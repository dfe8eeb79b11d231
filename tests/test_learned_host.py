"""Host-side pieces of the learned preconditioner's training code (CPU only)."""
import numpy as np


def test_initial_weights_are_jacobi(oracle_mod):
    """The initial network of the training code outputs L = I for any input."""
    from oracle import mlp
    from paper_2112_05598_amd.learned import init_weights
    rng = np.random.default_rng(0)
    feat = rng.normal(size=(20, mlp.N_IN)) * 10
    blocks = np.concatenate([rng.uniform(1, 2, (20, 1)), rng.uniform(-0.5, 0.5, (20, 3)), rng.uniform(1, 2, (20, 1))],
                            axis=1)
    L = mlp.factor(mlp.forward(init_weights(7), mlp.feature_stats(feat), feat, blocks)[0])
    np.testing.assert_allclose(L, np.broadcast_to(np.eye(4), L.shape), atol=1e-4)
