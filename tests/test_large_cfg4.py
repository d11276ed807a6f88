"""Sampled parity at the full size of cfg4 (diamond Fd-3m, non-symmorphic, 6^3 mesh, nao 52,
naux 300, ntau 128): FP64 and three-piece bfloat16 contractions (the two forms this workload
compares; steps in tests/fullsize_common.py)."""
import pytest

from tests.fullsize_common import compare, run, setup

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(900)]


@pytest.fixture(scope="module")
def cfg4():
    return setup("cfg4")


def test_cfg4_sampled_fp64(cfg4):
    compare(cfg4, *run(cfg4, 0), 1e-10)


def test_cfg4_sampled_bf16x6(cfg4):
    compare(cfg4, *run(cfg4, 2), 1e-6)
