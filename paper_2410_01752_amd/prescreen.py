"""Pre-screening of the base features on the GPU (Sec. 3.1, eq. mi-exact;
the initial screening option of Sec. 3.3): score every primary feature
against y by kernel-density mutual information or |Spearman correlation| and
keep the best ceil(quantile d) before expansion.  Argument marshalling only;
the scores and the selection are computed by the library's kernels."""
from __future__ import annotations

from typing import Tuple

import numpy as np
import torch

from . import _lib as L


def prescreen(X: np.ndarray, y: np.ndarray, method: str = "mi", quantile: float = 0.01,
              device: str = "cuda:0") -> Tuple[np.ndarray, np.ndarray]:
    """(kept feature indices by (score desc, index asc), all d scores)."""
    if method not in L.PRESCREEN:
        raise L.SissoError(f"unknown pre-screening method {method!r}")
    dev = torch.device(device)
    X = np.asarray(X, dtype=np.float64)
    n, d = X.shape
    Xd = torch.from_numpy(np.ascontiguousarray(X.T)).to(dev)
    yd = torch.from_numpy(np.ascontiguousarray(y, dtype=np.float64)).to(dev)
    sc = torch.empty(d, dtype=torch.float64, device=dev)
    lib = L.lib()
    nb = lib.sisso_prescreen_workspace_size(n, d)
    ws = torch.empty(max(nb, 256), dtype=torch.uint8, device=dev)
    st = L.stream_handle(dev)
    L.check(lib.sisso_prescreen_scores(L.ptr(Xd), n, n, d, L.ptr(yd), L.PRESCREEN[method], L.ptr(sc), L.ptr(ws),
                                       ws.numel(), st), "sisso_prescreen_scores")
    idx = torch.empty(d, dtype=torch.int32, device=dev)
    cnt = torch.zeros(1, dtype=torch.int32, device=dev)
    L.check(lib.sisso_prescreen_select(L.ptr(sc), d, float(quantile), L.ptr(idx), L.ptr(cnt), st),
            "sisso_prescreen_select")
    c = int(cnt.item())
    return idx[:c].cpu().numpy().astype(np.int64), sc.cpu().numpy()
