"""Network: a reusable contraction blueprint (Sec. "Network").

A network is defined by lines ``NAME: i, j, ...`` (one per tensor, the
index names are the network's own), ``TOUT: i, l`` (the output's index
order; ``;`` may separate row and column indices) and optionally
``ORDER: ((M1,M2),M3)``.  Tensors are loaded with :meth:`Network.put`,
which maps a tensor's own labels onto the network's index names, so the
same network serves tensors with any labels.  The contraction order is the
one given, or the optimum of the library's dynamic programming with cost
capping (``bst_network_order``), computed from the loaded dims.  Every
pairwise step runs as a block-sparse contraction plan on the GPU and a
final permute puts the output in TOUT order.
"""
from __future__ import annotations

import ctypes as C
import re
from typing import Dict, List, Sequence, Tuple

from . import bst


def _parse_order(s: str):
    """``((A,B),C)`` -> nested tuples of names."""
    tok = re.findall(r"\(|\)|,|[^(),\s]+", s)
    pos = 0

    def node():
        nonlocal pos
        if tok[pos] == "(":
            pos += 1
            left = node()
            if tok[pos] != ",":
                raise ValueError("ORDER: expected ','")
            pos += 1
            right = node()
            if tok[pos] != ")":
                raise ValueError("ORDER: expected ')'")
            pos += 1
            return (left, right)
        name = tok[pos]
        pos += 1
        return name

    tree = node()
    if pos != len(tok):
        raise ValueError("ORDER: trailing input")
    return tree


def _order_string(tree) -> str:
    return tree if isinstance(tree, str) else f"({_order_string(tree[0])},{_order_string(tree[1])})"


def _relabeled(T: bst.Tensor, labels: Sequence[str]) -> bst.Tensor:
    """A descriptor with T's legs (same order, charges, dims) and new labels."""
    sym = T.symmetry()
    _, legs = T.legs()
    if sym == [0]:
        return bst.Tensor(list(labels), legs)
    full = []
    for i, (d, secs) in enumerate(legs):
        qs = T.leg_charges(i)
        full.append((d, [(q if len(sym) > 1 else q[0], g) for q, (_, g) in zip(qs, secs)]))
    return bst.Tensor(list(labels), full, sym=sym)


class Network:
    def __init__(self, lines: Sequence[str]):
        self.names: List[str] = []
        self.indices: Dict[str, List[str]] = {}
        self.tout: List[str] = []
        self.order = None
        for raw in lines:
            line = raw.split("#", 1)[0].strip()
            if not line:
                continue
            key, _, rest = line.partition(":")
            key = key.strip()
            if key == "ORDER":
                self.order = _parse_order(rest.strip()) if rest.strip() else None
                continue
            labs = [l for l in re.split(r"[,;\s]+", rest.strip()) if l]
            if key == "TOUT":
                self.tout = labs
            else:
                if key in self.indices:
                    raise ValueError(f"tensor {key} defined twice")
                self.names.append(key)
                self.indices[key] = labs
        if not self.names:
            raise ValueError("a network needs at least one tensor")
        count: Dict[str, int] = {}
        for n in self.names:
            for l in self.indices[n]:
                count[l] = count.get(l, 0) + 1
        if any(c > 2 for c in count.values()):
            raise ValueError("an index joins more than two tensors")
        open_ = sorted(l for l, c in count.items() if c == 1)
        if sorted(self.tout) != open_:
            raise ValueError("TOUT must list exactly the open indices")
        self.tensors: Dict[str, bst.Tensor] = {}
        self.optimal = self.order is None

    @classmethod
    def from_string(cls, lines: Sequence[str]) -> "Network":
        return cls(lines)

    def put(self, name: str, T: bst.Tensor, labels: Sequence[str]):
        """Load T as tensor ``name``; ``labels`` lists T's labels in the order
        of the network's indices of ``name``."""
        if name not in self.indices:
            raise KeyError(name)
        net = self.indices[name]
        if len(labels) != len(net) or T.rank != len(net):
            raise ValueError(f"{name}: one label per index")
        own = T.labels
        if sorted(own) != sorted(labels):
            raise ValueError(f"{name}: labels do not match the tensor's")
        to_net = dict(zip(labels, net))
        self.tensors[name] = _relabeled(T, [to_net[l] for l in own])

    def set_order(self, optimal: bool = True, order: str | None = None):
        self.optimal = optimal
        if order is not None:
            self.order = _parse_order(order)
            self.optimal = False

    def get_order(self) -> str:
        return _order_string(self.order) if self.order is not None else ""

    def optimize(self) -> float:
        """Optimal order for the loaded dims (bst_network_order); its cost."""
        missing = [n for n in self.names if n not in self.tensors]
        if missing:
            raise ValueError(f"tensors not loaded: {missing}")
        ids: Dict[str, int] = {}
        dims: List[int] = []
        legs: List[int] = []
        for n in self.names:
            T = self.tensors[n]
            labels, tl = T.legs()
            for l, (_, secs) in zip(labels, tl):
                if l not in ids:
                    ids[l] = len(dims)
                    dims.append(sum(g for _, g in secs))
                legs.append(ids[l])
        k = len(self.names)
        nl = (C.c_int32 * k)(*[self.tensors[n].rank for n in self.names])
        lg = (C.c_int32 * max(len(legs), 1))(*legs)
        dm = (C.c_int64 * max(len(dims), 1))(*dims)
        pairs = (C.c_int32 * max(2 * (k - 1), 1))()
        cost = C.c_double()
        bst._check(bst.lib().bst_network_order(k, nl, lg, len(dims), dm, pairs, C.byref(cost)))
        nodes: List = list(self.names)
        for s in range(k - 1):
            nodes.append((nodes[pairs[2 * s]], nodes[pairs[2 * s + 1]]))
        self.order = nodes[-1]
        return cost.value

    def launch(self, buffers: Dict[str, object], prec="fp64", torch=None):
        """Contract the loaded tensors, whose data are ``buffers[name]``
        (device float64 tensors); returns (descriptor, device data) of the
        output in TOUT order."""
        if torch is None:
            import torch
        if self.optimal or self.order is None:
            self.optimize()
        dev = next(iter(buffers.values())).device

        def run(node):
            if isinstance(node, str):
                return self.tensors[node], buffers[node]
            (ta, a), (tb, b) = run(node[0]), run(node[1])
            tc, plan = bst.contract_plan(ta, tb, prec)
            out = torch.empty(max(tc.numel, 1), dtype=torch.float64, device=dev)[:tc.numel]
            plan.execute([a, b], [out], bst.workspace(plan.workspace_bytes, device=dev))
            return tc, out

        T, data = run(self.order)
        if T.labels != self.tout:
            tp, plan = bst.permute_plan(T, self.tout)
            out = torch.empty(max(tp.numel, 1), dtype=torch.float64, device=dev)[:tp.numel]
            plan.execute([data], [out], bst.workspace(plan.workspace_bytes, device=dev))
            T, data = tp, out
        return T, data
