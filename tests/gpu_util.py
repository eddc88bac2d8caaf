"""Helpers for the GPU parity tests: host<->device marshalling and oracle comparison."""
import numpy as np
import torch

import oracle

DEV = "cuda"


def d(a: np.ndarray) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def h(t: torch.Tensor) -> np.ndarray:
    return t.cpu().numpy()


def check_layout(table, kind):
    rc, st = oracle.check_layout(h(table.dump_slots()), table.windows, table.window, table.scheme, table.seed, kind)
    assert rc == 0, f"layout: {oracle.LAYOUT_ERRORS[rc]} at slot {st['first_bad_slot']}"
    return st
