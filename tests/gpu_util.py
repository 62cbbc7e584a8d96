"""Helpers shared by the GPU tests: device copies of generator instances and
the normwise error metric.

Error metric (nodal forces, displacements): e = max_n |A_n - B_n| / max_n |B_n|
with |.| the Euclidean norm of the node's 3-vector.
"""
import numpy as np
import torch

from paper_2005_02498_amd import workloads as W

MAT = {"mu": W.MU, "nu": W.NU, "a": W.CORE_A, "B": W.DRAG_B}


def dev(inst):
    d = torch.device("cuda:0")
    return dict(
        x=torch.tensor(inst.x, dtype=torch.float64, device=d).contiguous(),
        seg_nodes=torch.tensor(inst.seg_nodes, dtype=torch.int32, device=d).contiguous(),
        burgers=torch.tensor(inst.burgers, dtype=torch.float64, device=d).contiguous(),
        normal=torch.tensor(inst.normal, dtype=torch.float64, device=d).contiguous(),
        pinned=torch.tensor(inst.pinned, dtype=torch.uint8, device=d).contiguous(),
    )


def normwise(a, b):
    a = np.asarray(a); b = np.asarray(b)
    num = np.linalg.norm(a - b, axis=0).max()
    den = np.linalg.norm(b, axis=0).max()
    return float(num / den) if den > 0 else float(num)


def batch_dev(bt):
    d = torch.device("cuda:0")
    return dict(
        x=torch.tensor(bt.x, dtype=torch.float64, device=d).contiguous(),
        seg_nodes=torch.tensor(bt.seg_nodes, dtype=torch.int32, device=d).contiguous(),
        burgers=torch.tensor(bt.burgers, dtype=torch.float64, device=d).contiguous(),
        normal=torch.tensor(bt.normal, dtype=torch.float64, device=d).contiguous(),
        pinned=torch.tensor(bt.pinned, dtype=torch.uint8, device=d).contiguous(),
        sigma_app=torch.tensor(bt.sigma_app, dtype=torch.float64, device=d).contiguous(),
        volume=torch.tensor(bt.volume, dtype=torch.float64, device=d).contiguous(),
    )
