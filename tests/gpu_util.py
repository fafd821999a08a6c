"""Helpers shared by the GPU parity tests (no arithmetic of the method here)."""
import sys

import numpy as np
import torch

import paper_2307_16080_amd as mlk
from paper_2307_16080_amd import _lib as L


def dev(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def bits16(t):
    """bf16 tensor -> uint16 codes on the host."""
    torch.cuda.synchronize()
    return t.view(torch.int16).cpu().numpy().view(np.uint16)


def bits8(t):
    torch.cuda.synchronize()
    return t.view(torch.uint8).cpu().numpy()


def from_bf16_codes(codes):
    return torch.from_numpy(np.ascontiguousarray(codes).view(np.int16)).view(torch.bfloat16).cuda()


def from_e4m3_codes(codes):
    return torch.from_numpy(np.ascontiguousarray(codes)).view(torch.float8_e4m3fn).cuda()


def all_tiles(in_dtype, out_dtype, conv=False):
    """One configuration per compiled tile kernel of this dtype (split 1)."""
    if conv:
        p = mlk.conv_problem(64, 512, 64, 64, 512, 3, 3, 1, 1, in_dtype, out_dtype)
    else:
        p = mlk.matmul_problem(8192, 8192, 8192, in_dtype, out_dtype)
    seen, out = set(), []
    for c in mlk.configs(p):
        key = (c.bm, c.bn, c.bk, c.wm, c.wn, c.stages, c.layout, c.mfma)
        if key not in seen:
            seen.add(key)
            out.append(mlk.TileConfig(*key[:5], 1, 1, 0, key[5], key[6], key[7]))
    return out


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def normwise(c, r):
    d = np.asarray(c, np.float64) - np.asarray(r, np.float64)
    rn = np.linalg.norm(np.asarray(r, np.float64))
    return float(np.linalg.norm(d) / rn) if rn > 0 else float(np.linalg.norm(d))
