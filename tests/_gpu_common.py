"""Shared helpers of the GPU tests (not collected)."""
import numpy as np
import torch

import paper_2505_00715_amd as g
from oracle import freqmap


def make_ctx(xyz, tri, c, s, leaf, eta, sym=True):
    ctx = g.Context(0)
    ctx.upload_mesh(xyz, tri, c)
    ctx.set_frequencies(s, sym)
    ctx.build_cluster_tree(leaf, eta)
    return ctx


def to_dev(X, prec):
    dt = torch.complex128 if prec == g.C128 else torch.complex64
    return torch.from_numpy(np.ascontiguousarray(X)).to(dt).cuda()


def from_dev(t):
    torch.cuda.synchronize()
    return t.cpu().numpy().astype(np.complex128)


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def kpos_map(s):
    rep, conj = freqmap.representatives(s)
    K = freqmap.distinct(rep)
    return rep, conj, K, {int(k): p for p, k in enumerate(K)}
