"""ADAM recurrence (oracle; test infrastructure).

The paper minimises the SCA potential with PyTorch's ADAM optimizer (Sec. II
after Eq. (7); Sec. III); it states no hyper-parameters.  This is Kingma & Ba,
"Adam: a method for stochastic optimization" (ICLR 2015), Algorithm 1,
with PyTorch's defaults where the paper is silent (eps = 1e-8, no weight
decay, no AMSGrad):

  t <- t + 1
  m <- b1 m + (1 - b1) g
  v <- b2 v + (1 - b2) g^2
  x <- x - lr * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps)

Pinned against torch.optim.Adam on the CPU fed the same gradients.
"""
from __future__ import annotations

import dataclasses

import numpy as np


@dataclasses.dataclass
class AdamState:
    m: np.ndarray
    v: np.ndarray
    t: int = 0

    @classmethod
    def zeros(cls, n: int) -> "AdamState":
        return cls(np.zeros(n), np.zeros(n), 0)


def adam_step(x: np.ndarray, g: np.ndarray, st: AdamState, lr: float,
              b1: float = 0.9, b2: float = 0.999, eps: float = 1e-8):
    """One ADAM update; returns the new x (st is updated in place)."""
    st.t += 1
    st.m = b1 * st.m + (1.0 - b1) * g
    st.v = b2 * st.v + (1.0 - b2) * g * g
    mhat = st.m / (1.0 - b1 ** st.t)
    vhat = st.v / (1.0 - b2 ** st.t)
    return x - lr * mhat / (np.sqrt(vhat) + eps)
