"""Host logic of the training loop: the epoch schedule of the temporal-
visibility lifecycle (Sec. 3.3) and the optimiser."""

import torch

from paper_2503_08217_amd.train import Adam, epoch_action


def test_fold_every_epoch_reset_periodically():
    acts = [epoch_action(e, 3) for e in range(7)]
    assert acts == ["fold", "fold", "reset", "fold", "fold", "reset", "fold"]
    assert all(epoch_action(e, 0) == "fold" for e in range(5))


def test_adam_minimises_a_quadratic():
    x = torch.tensor([3.0, -2.0, 0.5], dtype=torch.float64)
    target = torch.tensor([1.0, 1.0, 1.0], dtype=torch.float64)
    opt = Adam(dict(x=0.05))
    for _ in range(400):
        g = 2 * (x - target)
        opt.step(dict(x=x), dict(x=g))
    assert torch.allclose(x, target, atol=1e-2)
