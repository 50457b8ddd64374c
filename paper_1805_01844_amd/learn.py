"""Training and evaluation of the learned class selector (GPU, through the library's kernels).

Labels come from exhaustive search: for every block the library's feature kernel returns
its 19 features, the words of all 16 classes and the smallest class (ties to the lowest id).
The network is trained with the library's loss/gradient and Adam kernels; PyTorch only holds
the tensors, shuffles sample indices and gathers mini-batches.

The trained parameters ship next to this module (``selector.f32``: 2320 little-endian
binary32 values, ``selector.json``: how they were made); ``load_selector()`` reads them.
"""
from __future__ import annotations

import json
import os
import time

import numpy as np
import torch

import paper_1805_01844_amd as pc

HERE = os.path.dirname(os.path.abspath(__file__))
MODEL_PATH = os.path.join(HERE, "selector.f32")
META_PATH = os.path.join(HERE, "selector.json")
BLOCK_LENS = (256, 512, 1024, 4096)
_GROUP = {1: 0, 2: 1, 4: 2}


def load_selector(path: str = MODEL_PATH) -> torch.Tensor:
    """The shipped parameters as a CPU float32 tensor (raises if the file is missing)."""
    a = np.fromfile(path, dtype="<f4")
    if a.size != pc.MLP_PARAMS:
        raise ValueError("%s: %d floats, expected %d" % (path, a.size, pc.MLP_PARAMS))
    return torch.from_numpy(a.astype(np.float32))


def use_selector(path: str = MODEL_PATH) -> torch.Tensor:
    """Loads the shipped parameters into the library on the current device."""
    p = load_selector(path)
    pc.set_model(p)
    return p


def save_selector(params: torch.Tensor, meta: dict, path: str = MODEL_PATH, meta_path: str = META_PATH) -> None:
    params.detach().cpu().numpy().astype("<f4").tofile(path)
    with open(meta_path, "w") as f:
        json.dump(meta, f, indent=1, sort_keys=True)


def dataset(segments, block_len_of) -> tuple:
    """(X [N, 19] float32, labels [N] u8, class words [N, 16] int32 with -1 for invalid) over
    every block of the segments; block_len_of(i, segment) gives each segment's block length."""
    xs, ys, ws = [], [], []
    for i, s in enumerate(segments):
        if s.numel() == 0:
            continue
        x, w, y = pc.block_features(s, block_len_of(i, s))
        xs.append(x)
        ys.append(y)
        ws.append(w)
    return torch.cat(xs), torch.cat(ys), torch.cat(ws)


def init_params(seed: int, device="cuda") -> torch.Tensor:
    """He-style uniform initialisation, zero biases."""
    g = torch.Generator(device="cpu")
    g.manual_seed(seed)
    w1 = (torch.rand(64, 19, generator=g, dtype=torch.float64) * 2 - 1) * (6.0 / 19) ** 0.5
    w2 = (torch.rand(16, 64, generator=g, dtype=torch.float64) * 2 - 1) * (6.0 / 64) ** 0.5
    p = torch.cat([w1.reshape(-1), torch.zeros(64, dtype=torch.float64), w2.reshape(-1),
                   torch.zeros(16, dtype=torch.float64)])
    return p.to(torch.float32).to(device)


def train(X: torch.Tensor, y: torch.Tensor, epochs: int = 10, batch: int = 8192, lr: float = 3e-3, seed: int = 0,
          params: torch.Tensor = None, log=None):
    """Adam on mini-batches of shuffled samples. Returns (params, per-epoch mean losses)."""
    dev = X.device
    p0 = init_params(seed, dev) if params is None else params
    tr = pc.MLPTrainer(p0, batch, lr=lr)
    g = torch.Generator(device=dev)
    g.manual_seed(seed)
    n = X.shape[0]
    hist = []
    for ep in range(epochs):
        perm = torch.randperm(n, generator=g, device=dev)
        tot, cnt = torch.zeros((), device=dev), 0
        for b0 in range(0, n - batch + 1, batch):
            idx = perm[b0:b0 + batch]
            tr.step(X.index_select(0, idx).contiguous(), y.index_select(0, idx).contiguous())
            tot += tr.loss[0]
            cnt += 1
        hist.append(float(tot.item()) / max(cnt, 1))
        if log:
            log("epoch %d loss %.4f" % (ep, hist[-1]))
    return tr.params, hist


def choose(params: torch.Tensor, X: torch.Tensor, words: torch.Tensor) -> torch.Tensor:
    """Classes the selector keeps: the first top score, replaced by class 0 when invalid or
    not strictly smaller than class 0 (the rule of the compressor)."""
    pred = torch.argmax(pc.mlp_scores(params, X), dim=1)  # first maximal index
    wp = words.gather(1, pred.reshape(-1, 1)).reshape(-1)
    keep = (wp != -1) & (wp < words[:, 0])
    return torch.where(keep, pred, torch.zeros_like(pred))


def payload_words(params: torch.Tensor, X: torch.Tensor, y: torch.Tensor, words: torch.Tensor) -> dict:
    """Payload words of the plain (class 0), learned and exhaustive choices, and the
    learned top-1 agreement with the exhaustive label."""
    w64 = words.to(torch.int64)
    cls = choose(params, X, words)
    return {
        "plain": int(w64[:, 0].sum().item()),
        "learned": int(w64.gather(1, cls.reshape(-1, 1)).sum().item()),
        "exhaustive": int(w64.gather(1, y.to(torch.int64).reshape(-1, 1)).sum().item()),
        "agreement": float((torch.argmax(pc.mlp_scores(params, X), dim=1) == y.to(torch.int64)).float().mean()),
    }


def _events(n_events: int, seed: int, device):
    import datagen  # seeded synthetic inputs (repository root)

    return [e.reshape(-1) for e in datagen.uneven_events(n_events, seed=seed, device=device)]


def main(n_blocks: int = 1_000_000, seed: int = 100, test_seed: int = 200, epochs: int = 12, out_dir: str = None):
    """Trains on at least n_blocks blocks of uneven camera events (block lengths cycling through
    BLOCK_LENS), evaluates on held-out events, writes the parameters and a summary."""
    dev = "cuda"
    pc.init()
    t0 = time.time()
    segs, tot = [], 0
    i = 0
    while tot < n_blocks:
        ev = _events(64, seed + i, dev)
        for s in ev:
            L = BLOCK_LENS[len(segs) % len(BLOCK_LENS)]
            segs.append((s, L))
            tot += (s.numel() + L - 1) // L
        i += 1
    X, y, W = dataset([s for s, _ in segs], lambda k, s: segs[k][1])
    del segs
    X, y, W = X[:n_blocks].contiguous(), y[:n_blocks].contiguous(), W[:n_blocks].contiguous()
    t1 = time.time()
    params, hist = train(X, y, epochs=epochs, log=lambda m: print(m, flush=True))
    t2 = time.time()
    ev = _events(256, test_seed, dev)
    Xt, yt, Wt = dataset(ev, lambda k, s: BLOCK_LENS[k % len(BLOCK_LENS)])
    res_train = payload_words(params, X, y, W)
    res_test = payload_words(params, Xt, yt, Wt)
    meta = {
        "training_blocks": int(X.shape[0]), "training_seed": seed, "test_seed": test_seed,
        "block_lens": list(BLOCK_LENS), "epochs": epochs, "batch": 8192, "lr": 3e-3, "optimizer": "adam",
        "loss_per_epoch": hist, "train": res_train, "test": res_test,
        "data": "uneven camera events: shapes 1855x40, 2048x96, 11328x128; u16/u32; noise sigma U(2,20); "
                "pulse fraction U(0,5%)",
        "seconds": {"data": t1 - t0, "train": t2 - t1},
    }
    if out_dir:
        os.makedirs(out_dir, exist_ok=True)
        save_selector(params, meta, os.path.join(out_dir, "selector.f32"), os.path.join(out_dir, "selector.json"))
    else:
        save_selector(params, meta)
    print(json.dumps({"train": res_train, "test": res_test, "loss": hist[-1]}), flush=True)
    return params, meta


if __name__ == "__main__":
    import sys

    main(out_dir=sys.argv[1] if len(sys.argv) > 1 else None)
