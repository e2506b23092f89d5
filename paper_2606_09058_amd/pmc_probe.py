"""Workload for the memory-traffic counters of the tridiagonalisation's
symmetric product, to be run under rocprofv3 once per counter:

    rocprofv3 --pmc FETCH_SIZE -d <dir> -f csv -- python3 <repo>/paper_2606_09058_amd/pmc_probe.py
    rocprofv3 --pmc WRITE_SIZE -d <dir> -f csv -- python3 <repo>/paper_2606_09058_amd/pmc_probe.py

It first fills and then copies a 1 GiB device buffer (a plain copy of known
size: the fill writes 1 GiB, the copy reads 1 GiB and writes 1 GiB), whose
counter values give the scale of each counter, and then runs one FP64 solve
(ks_gevd, all eigenvectors) of the N = 6656 supercell workload, whose
symv_kernel dispatches are the ones measured.  Prints what it ran.
"""
import os
import sys

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

import numpy as np  # noqa: E402
import torch  # noqa: E402

from paper_2606_09058_amd import inputs as I  # noqa: E402
from paper_2606_09058_amd import ks  # noqa: E402

COPY_BYTES = 1 << 30


def main():
    assert torch.cuda.is_available(), "needs a GPU"
    x = torch.empty(COPY_BYTES // 8, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    x.fill_(1.0)
    y.copy_(x)
    torch.cuda.synchronize()
    print("copy_bytes", COPY_BYTES, flush=True)
    del x, y
    p = I.workload(sys.argv[1] if len(sys.argv) > 1 else "supercell6656")
    plan = ks.Plan(p.n, complex=np.iscomplexobj(p.H), noncollinear=p.nsp == 2)
    H = torch.from_numpy(p.H).cuda()
    S = torch.from_numpy(p.S.astype(p.H.dtype)).cuda()
    eps = torch.empty(plan._vshape(), dtype=torch.float64, device="cuda")
    C = torch.empty(plan._mshape(), dtype=plan.mdtype, device="cuda")
    plan.gevd(H, S, eps, C)
    plan.check("probe solve")
    print("solved", p.name, "order", p.order, flush=True)


if __name__ == "__main__":
    main()
