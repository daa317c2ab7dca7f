"""Helpers for the GPU parity tests: run the HIP path through the C-ABI binding
and compare with the oracle on the same seeded inputs."""
import numpy as np

import oracle as O


def device():
    import torch
    return torch.device("cuda:0")


def to_dev(edges):
    import torch
    e = np.ascontiguousarray(edges, dtype=np.int64).reshape(-1, 2)
    return torch.from_numpy(e).to(device())


class Case:
    """One graph on both sides: device CSR (HIP) and oracle CSR + labels."""

    def __init__(self, edges, n):
        import paper_2012_13548_amd as g5
        self.edges = np.ascontiguousarray(edges, dtype=np.int64).reshape(-1, 2)
        self.n = n
        self.csr = g5.build_csr(to_dev(self.edges), n)
        self.ocsr = O.build_csr(self.edges, n)
        self.label = O.components(self.edges, n)

    def check_csr(self):
        rp, ci = self.csr.arrays()
        assert np.array_equal(rp.cpu().numpy(), self.ocsr.row_ptr)
        assert np.array_equal(ci.cpu().numpy(), self.ocsr.col_idx)

    def check_root(self, root, **kw):
        import paper_2012_13548_amd as g5
        parent, level, st = g5.bfs(self.csr, root, stats=True, **kw)
        parent, level = parent.cpu().numpy(), level.cpu().numpy()
        # every reached vertex was claimed exactly once (queue and bitmap counts)
        assert st["reached"] == int((level >= 0).sum()), (root, kw, st["reached"])
        _, olevel = O.bfs(self.ocsr, root)
        bad = np.flatnonzero(level != olevel)
        assert bad.size == 0, (f"root {root} {kw}: {bad.size} levels differ, first at "
                               f"{bad[:5]}: gpu {level[bad[:5]]} oracle {olevel[bad[:5]]}")
        rule = O.validate(self.ocsr, root, parent, level, self.label)
        assert rule == 0, f"root {root} {kw}: parent array invalid ({O.RULES[rule]})"
        return parent, level


def check_batch(case, roots, **kw):
    """g5_bfs_batch rows vs the oracle: levels bit-exact (int8), parents valid."""
    import paper_2012_13548_amd as g5
    want_par = kw.pop("parents", True)
    res = g5.bfs_batch(case.csr, roots, parents=want_par, stats=True, **kw)
    parents, levels, info = res
    levels = levels.cpu().numpy()
    parents = parents.cpu().numpy() if parents is not None else None
    for b, r in enumerate(roots):
        _, olevel = O.bfs(case.ocsr, r)
        bad = np.flatnonzero(levels[b].astype(np.int32) != olevel)
        assert bad.size == 0, (f"batch row {b} root {r} {kw}: {bad.size} levels differ, first "
                               f"{bad[:5]}: gpu {levels[b][bad[:5]]} oracle {olevel[bad[:5]]}")
        if parents is not None:
            rule = O.validate(case.ocsr, r, parents[b], olevel, case.label)
            assert rule == 0, f"batch row {b} root {r} {kw}: parents invalid ({O.RULES[rule]})"
    return parents, levels, info
