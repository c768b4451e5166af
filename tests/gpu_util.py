"""Helpers for GPU tests: skip cleanly without a GPU, load the built library."""
import os
import sys

import pytest
import torch


def require_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2402_18008_amd import _abi
    if not os.path.exists(_abi.LIB_PATH):
        pytest.fail("libhomog.so is not built (run __graft_entry__.build() first)")
    _abi.lib()


def announce(msg):
    """Name the case before a GPU step (flushed, so it survives a crash)."""
    sys.stdout.write(f"\n[gpu] {msg}\n")
    sys.stdout.flush()
