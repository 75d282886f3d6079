"""Oracle of the merged time grid of a prediction.

TEST INFRASTRUCTURE ONLY. Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import or call anything here; the GPU
library shares no code with it.

The paper predicts at test times by adding them to the state-space model as
steps without a measurement (missing-measurement elements, section 3) and
running filter and smoother over the sorted union of training and test times
(section 4). The union is the stable merge of the two sorted sequences:
at equal times a training step precedes a test step, and each sequence keeps
its own order. Written out as ranks, the merged index of
  training element i  is  i + #{j : t_test[j] <  t_train[i]},
  test element j      is  j + #{i : t_train[i] <= t_test[j]},
which is what this module computes (numpy's searchsorted counts the set).
"""
from __future__ import annotations

import numpy as np


def merge_ranks(t_train, t_test):
    """Merged index of every training and every test element (int64)."""
    t_train = np.asarray(t_train, np.float64)
    t_test = np.asarray(t_test, np.float64)
    pos_train = np.arange(t_train.shape[0], dtype=np.int64) + np.searchsorted(t_test, t_train, side="left")
    pos_test = np.arange(t_test.shape[0], dtype=np.int64) + np.searchsorted(t_train, t_test, side="right")
    return pos_train, pos_test


def merge_times(t_train, y_train, t_test, mask_train=None):
    """(t, y, mask, test_pos) of the merged grid: y_train at training steps
    and 0 at test steps (y is None when y_train is None), mask_train (or 1)
    at training steps and 0 at test steps, test_pos the merged index of
    every test time."""
    t_train = np.asarray(t_train, np.float64)
    t_test = np.asarray(t_test, np.float64)
    n, m = t_train.shape[0], t_test.shape[0]
    pos_train, pos_test = merge_ranks(t_train, t_test)
    t = np.empty(n + m, np.float64)
    t[pos_train] = t_train
    t[pos_test] = t_test
    mask = np.zeros(n + m, np.uint8)
    mask[pos_train] = 1 if mask_train is None else np.asarray(mask_train, np.uint8)
    y = None
    if y_train is not None:
        y_train = np.asarray(y_train)
        y = np.zeros(n + m, y_train.dtype)
        y[pos_train] = y_train
    return t, y, mask, pos_test
