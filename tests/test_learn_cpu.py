"""Host-side pieces of the learned ordering: parameter layout and the top-q recall metric."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_1812_08491_amd import learn  # noqa: E402
from paper_1812_08491_amd._lib import PC_MLP_PARAMS  # noqa: E402


def test_init_params_layout():
    p = learn.init_params(np.random.default_rng(0))
    assert p.shape == (PC_MLP_PARAMS,) and p.dtype == np.float32
    # biases b1 (after W1), b2 (after W2) and b3 (last) start at zero
    assert not p[512:576].any() and not p[576 + 4096:576 + 4096 + 64].any() and p[-1] == 0
    assert p[:512].std() > 0.3 and p[576:576 + 4096].std() > 0.1


def test_topq_recall_by_hand():
    # direction 7: candidates scored 0.9 (pos), 0.5, 0.1 (pos) -> positives at ranks 0 and 2
    # direction 3: 0.2 (neg), 0.8 (pos)                          -> positive at rank 0
    scores = torch.tensor([0.9, 0.5, 0.1, 0.2, 0.8])
    labels = torch.tensor([1.0, 0.0, 1.0, 0.0, 1.0])
    direction = torch.tensor([7, 7, 7, 3, 3])
    assert learn.topq_recall(scores, labels, direction, 1) == 0.5
    assert learn.topq_recall(scores, labels, direction, 2) == 0.5
    assert learn.topq_recall(scores, labels, direction, 3) == 1.0
    # ties are broken by row order, so equal scores rank the earlier candidate first
    tied = torch.tensor([0.5, 0.5])
    assert learn.topq_recall(tied, torch.tensor([0.0, 1.0]), torch.tensor([1, 1]), 1) == 0.0
    assert learn.topq_recall(tied, torch.tensor([1.0, 0.0]), torch.tensor([1, 1]), 1) == 1.0
