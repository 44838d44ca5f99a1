"""Host logic of the path workflow (no GPU): upsampling indices, segment
cutting and assembly."""
import numpy as np
import pytest
import torch

from paper_2605_26016_amd import mep


@pytest.mark.parametrize("n_old,n_new", [(3, 3), (3, 9), (5, 6), (4, 17), (2, 2), (2, 7)])
def test_upsample_indices_keep_every_image_in_order(n_old, n_new):
    idx = mep.upsample_indices(n_old, n_new)
    assert len(idx) == n_new and idx[0] == 0 and idx[-1] == n_old - 1
    assert np.all(np.diff(idx) >= 0) and np.all(np.diff(idx) <= 1)
    assert set(idx.tolist()) == set(range(n_old))


def test_upsample_needs_more_slots():
    with pytest.raises(ValueError):
        mep.upsample_indices(5, 4)


def test_split_and_assemble_round_trip():
    path = torch.arange(11 * 3 * 4, dtype=torch.float64).reshape(11, 3, 4)
    segs = mep.split(path, [0, 4, 7, 10])
    assert [s.shape[0] for s in segs] == [5, 4, 4]
    assert torch.equal(segs[0][-1], segs[1][0]) and torch.equal(segs[1][-1], segs[2][0])
    assert torch.equal(mep.assemble(segs), path)


def test_split_rejects_bad_cuts_and_assemble_rejects_gaps():
    path = torch.zeros(8, 3, 2, dtype=torch.float64)
    for cuts in ([1, 7], [0, 6], [0, 1, 7], [0, 4, 5, 7]):
        with pytest.raises(ValueError):
            mep.split(path, cuts)
    a, b = torch.zeros(3, 3, 2), torch.ones(3, 3, 2)
    with pytest.raises(ValueError):
        mep.assemble([a, b])
