"""Sampled parity at the full size of cfg2 (rocksalt Fm-3m, 6^3 mesh, nao 52, naux 250,
ntau 100): FP64, FP32 and three-piece bfloat16 contractions (steps in tests/fullsize_common.py)."""
import pytest

from tests.fullsize_common import compare, run, setup

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(900)]


@pytest.fixture(scope="module")
def cfg2():
    return setup("cfg2")


def test_cfg2_sampled_fp64(cfg2):
    compare(cfg2, *run(cfg2, 0), 1e-10)


def test_cfg2_sampled_fp32(cfg2):
    compare(cfg2, *run(cfg2, 1), 1e-6)


def test_cfg2_sampled_bf16x6(cfg2):
    compare(cfg2, *run(cfg2, 2), 1e-6)
