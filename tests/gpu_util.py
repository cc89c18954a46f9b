"""Helpers shared by the GPU parity tests (no method arithmetic here)."""
import sys

import numpy as np
import pytest
import torch


def have_gpu() -> bool:
    return torch.cuda.is_available()


def dev(a: np.ndarray) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t: torch.Tensor) -> np.ndarray:
    torch.cuda.synchronize()
    return t.cpu().numpy()


def announce(msg: str) -> None:
    """Name the GPU case before it runs (a fault can cut the log short)."""
    print(f"\n[gpu case] {msg}", flush=True)
    sys.stdout.flush()


def psnr(ref: np.ndarray, test: np.ndarray) -> float:
    d = ref.astype(np.float64) - test.astype(np.float64)
    mse = float(np.mean(d * d))
    return 99.99 if mse == 0 else 10.0 * np.log10(255.0 ** 2 / mse)


@pytest.fixture(scope="module")
def ctx():
    if not have_gpu():
        pytest.skip("no GPU")
    import paper_1311_1419_amd as P
    c = P.Context(0)
    yield c
    torch.cuda.synchronize()
    c.close()
