"""Plain-PyTorch NEP with autograd force training (forces by create_graph, then
a double backward for the parameter gradient) — the comparator the
hand-written adjoint is measured against, and an independent CPU cross-check
of the oracle's gradient. Shares no code with the oracle or the HIP library."""

from .nep_autograd import AutogradNEP, pairs_from_csr  # noqa: F401
