"""The round-trip that ``__graft_entry__.smoke()`` runs (one tiny step in FP64 and FP32
against the oracle), kept under test so that a change to the binding cannot leave it
broken."""

import os
import sys

import pytest

pytestmark = pytest.mark.gpu

pytest.importorskip("torch")


def test_smoke_entry_point():
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import __graft_entry__
    __graft_entry__.smoke()
