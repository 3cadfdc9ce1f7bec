"""Host checks of the seeded input recipes (no GPU)."""
import numpy as np
import pytest
import torch

import nys_inputs as ni


@pytest.mark.parametrize("n,p", [(256, 128), (128, 128)])
def test_device_ridge_generator_equals_host_recipe(n, p):
    """ridge_problem_device (run here on torch's CPU device) builds the same X and y as
    the numpy recipe from the same seed."""
    pr = ni.ridge_problem(n, p, 2.0, seed=3)
    X, y = ni.ridge_problem_device(n, p, 2.0, 3, torch.device("cpu"))
    assert np.max(np.abs(X.numpy() - pr.X)) <= 1e-15
    assert np.max(np.abs(y.numpy() - pr.y)) <= 1e-15
