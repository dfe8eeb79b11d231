"""Host-side pieces of the learned preconditioner's training code (CPU only)."""
import numpy as np


def test_fold_normalisation_matches_standardised_inputs(oracle_mod):
    """A network trained on (f - mu) / sd and folded into its first layer gives the same
    outputs on raw features f."""
    from oracle import mlp
    from paper_2112_05598_amd.learned import fold_normalisation, init_weights
    rng = np.random.default_rng(4)
    w = init_weights(2)
    p = mlp.unpack(w)
    p["W3"][:10] = rng.normal(0, 0.2, (10, 64))
    p["b1"][:] = rng.normal(0, 0.3, 64)
    w = mlp.pack(p)
    feat = rng.normal(size=(50, 12)) * rng.uniform(0.1, 20, 12) + rng.uniform(-30, 5, 12)
    mu, sd = feat.mean(0), feat.std(0)
    ref, _ = mlp.forward(w, (feat - mu) / sd)
    got, _ = mlp.forward(fold_normalisation(w, mu, sd), feat)
    np.testing.assert_allclose(got, ref, rtol=1e-9, atol=1e-9)


def test_initial_weights_are_jacobi(oracle_mod):
    """The initial network of the training code outputs L = I for any input."""
    from oracle import mlp
    from paper_2112_05598_amd.learned import init_weights
    feat = np.random.default_rng(0).normal(size=(20, 12)) * 10
    L = mlp.factor(mlp.forward(init_weights(7), feat)[0])
    np.testing.assert_allclose(L, np.broadcast_to(np.eye(4), L.shape), atol=1e-4)
