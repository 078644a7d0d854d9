"""The paper's graph summary models as presets of one refinement step.

Sec. "Graph Summaries for Bisimulation" expresses the summaries of Schätzle
et al. and Kaushik et al. in one parameterised model (models gsm:schaetzle
and gsm:kaushik).  With the step implemented here (vertex labels in P0,
(edge label, target block) pairs in the signature), each is a choice of
inputs:

* ``schaetzle``: forward, edge labels, no vertex labels (P0 = {V}, the
  initialisation of Alg. schaetzle-alg);
* ``kaushik``: backward (the transposed graph), vertex labels, no edge
  labels (Alg. kaushik-alg refines by incoming edges, starting from the
  label partition);
* ``full``: vertex and edge labels, forward or backward.

Each returns a ``Refiner`` bound to the prepared device graph.
"""
from __future__ import annotations

from typing import Optional

import torch

from . import Refiner, transpose


def schaetzle(row_ptr: torch.Tensor, col: torch.Tensor, elabel: Optional[torch.Tensor], kmax: int = 10,
              **kw) -> Refiner:
    """Edge-labelled forward bisimulation from P0 = {V}."""
    return Refiner(row_ptr, col, elabel, None, None, kmax=kmax, **kw)


def kaushik(row_ptr: torch.Tensor, col: torch.Tensor, vlabel: Optional[torch.Tensor],
            vlabel_ptr: Optional[torch.Tensor] = None, kmax: int = 10, **kw) -> Refiner:
    """Vertex-labelled backward bisimulation: the transposed graph, no edge labels."""
    rp_t, col_t, _ = transpose(row_ptr, col, None)
    return Refiner(rp_t, col_t, None, vlabel, vlabel_ptr, kmax=kmax, **kw)


def full(row_ptr: torch.Tensor, col: torch.Tensor, elabel: Optional[torch.Tensor], vlabel: Optional[torch.Tensor],
         vlabel_ptr: Optional[torch.Tensor] = None, direction: str = "fw", kmax: int = 10, **kw) -> Refiner:
    """Vertex- and edge-labelled bisimulation, forward ("fw") or backward ("bw")."""
    if direction == "bw":
        row_ptr, col, elabel = transpose(row_ptr, col, elabel)
    elif direction != "fw":
        raise ValueError("direction must be 'fw' or 'bw'")
    return Refiner(row_ptr, col, elabel, vlabel, vlabel_ptr, kmax=kmax, **kw)
