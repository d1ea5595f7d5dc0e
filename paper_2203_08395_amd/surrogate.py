"""Python binding of the RC-tree / learned-surrogate entry points of libsta.so.

Argument marshalling and the host side of training (mini-batch order, learning-rate
schedule, checkpoint files); every computation runs in the library's HIP kernels.  The
network, its features and the fallback rule are those of ``include/sta_surrogate.h``.
"""
from __future__ import annotations

import ctypes
import json
import math
import os

import numpy as np

from .sta import _P, _check, _ptr, _stream, load_library

N_PARAMS = 5378
OFF = {"W1": (0, (64, 16)), "b1": (1024, (64,)), "W2": (1088, (64, 64)), "b2": (5184, (64,)),
       "W3": (5248, (2, 64)), "b3": (5376, (2,))}
CAL_BINS, CAL_BUCKETS = 64, 128
TREE_ERR = {1: "net size", 2: "parent index", 4: "sink node"}


class TreesC(ctypes.Structure):
    _fields_ = [("n_nets", ctypes.c_int32), ("n_sinks", ctypes.c_int32), ("net_node_ptr", _P),
                ("node_parent", _P), ("node_R", _P), ("node_C", _P), ("sink_ptr", _P), ("sink_node", _P),
                ("sink_pincap", _P), ("drv_slew", _P), ("sink_net", _P)]


class AdamC(ctypes.Structure):
    _fields_ = [("lr", ctypes.c_float), ("beta1", ctypes.c_float), ("beta2", ctypes.c_float),
                ("eps", ctypes.c_float), ("step", ctypes.c_int32)]


_bound = False


def _lib():
    global _bound
    lib = load_library()
    if not _bound:
        T = ctypes.POINTER(TreesC)
        sz = ctypes.c_size_t
        lib.sta_tree_dataset.argtypes = [T, _P, _P, _P, _P, _P, _P]
        lib.sta_tree_exact.argtypes = [T, _P, _P, _P, _P, _P, _P]
        lib.sta_tree_features.argtypes = [T, _P, _P, _P]
        lib.sta_mlp_norm_scratch_bytes.argtypes = []
        lib.sta_mlp_norm_scratch_bytes.restype = sz
        lib.sta_mlp_norm.argtypes = [_P, ctypes.c_int32, _P, _P, sz, _P]
        lib.sta_mlp_grad_scratch_bytes.argtypes = [ctypes.c_int32]
        lib.sta_mlp_grad_scratch_bytes.restype = sz
        lib.sta_mlp_train_step.argtypes = [_P, _P, _P, ctypes.POINTER(AdamC), _P, _P, _P, _P, ctypes.c_int32, _P,
                                           _P, sz, _P]
        lib.sta_mlp_predict.argtypes = [_P, _P, _P, ctypes.c_int32, _P, _P]
        lib.sta_surrogate_cal_scratch_bytes.argtypes = []
        lib.sta_surrogate_cal_scratch_bytes.restype = sz
        lib.sta_surrogate_calibrate.argtypes = [_P, _P, _P, ctypes.c_int32, ctypes.c_double, ctypes.c_int32, _P,
                                                _P, sz, _P]
        lib.sta_surrogate_eval.argtypes = [T, _P, _P, _P, _P, ctypes.c_float, _P, _P, _P, _P, _P, _P, _P, _P]
        for f in ("sta_tree_dataset", "sta_tree_exact", "sta_tree_features", "sta_mlp_norm", "sta_mlp_train_step", "sta_mlp_predict",
                  "sta_surrogate_calibrate", "sta_surrogate_eval"):
            getattr(lib, f).restype = ctypes.c_int
        _bound = True
    return lib


EXPORTS = ("sta_tree_dataset", "sta_tree_exact", "sta_tree_features", "sta_mlp_norm_scratch_bytes", "sta_mlp_norm",
           "sta_mlp_grad_scratch_bytes", "sta_mlp_train_step", "sta_mlp_predict", "sta_surrogate_cal_scratch_bytes",
           "sta_surrogate_calibrate", "sta_surrogate_eval")


class Trees:
    """A set of RC-tree nets resident on the device (see ``sta_trees``)."""

    def __init__(self, T, device="cuda"):
        import torch
        self.device = torch.device(device)
        self.n_nets, self.n_sinks = int(T.n_nets), int(T.n_sinks)
        sink_net = np.repeat(np.arange(self.n_nets, dtype=np.int32), np.diff(T.sink_ptr))
        def dev(a, dt):
            return torch.from_numpy(np.ascontiguousarray(a, dtype=dt)).to(self.device)
        self.t = {"net_node_ptr": dev(T.net_node_ptr, np.int32), "node_parent": dev(T.node_parent, np.int32),
                  "node_R": dev(T.node_R, np.float32), "node_C": dev(T.node_C, np.float32),
                  "sink_ptr": dev(T.sink_ptr, np.int32), "sink_node": dev(T.sink_node, np.int32),
                  "sink_pincap": dev(T.sink_pincap, np.float32), "drv_slew": dev(T.drv_slew, np.float32),
                  "sink_net": dev(sink_net, np.int32)}
        self.status = torch.zeros(1, dtype=torch.int32, device=self.device)
        self.c = TreesC(self.n_nets, self.n_sinks, *[_ptr(self.t[k]) for k in
                                                     ("net_node_ptr", "node_parent", "node_R", "node_C", "sink_ptr",
                                                      "sink_node", "sink_pincap", "drv_slew", "sink_net")])

    def stream(self):
        import torch
        return _stream(torch, self.device)

    def check_status(self):
        """Raise if a kernel flagged a data error (synchronizes)."""
        v = int(self.status.item())
        if v:
            raise ValueError("RC-tree data error: " + ", ".join(n for b, n in TREE_ERR.items() if v & b))


def dataset(tr: Trees):
    """Features [S][12], targets [S][2], exact delay [S] and slew [S] (device tensors)."""
    import torch
    S = tr.n_sinks
    out = {"feat": torch.empty((S, 12), dtype=torch.float32, device=tr.device),
           "target": torch.empty((S, 2), dtype=torch.float32, device=tr.device),
           "delay": torch.empty(S, dtype=torch.float32, device=tr.device),
           "slew": torch.empty(S, dtype=torch.float32, device=tr.device)}
    _check(_lib().sta_tree_dataset(ctypes.byref(tr.c), _ptr(out["feat"]), _ptr(out["target"]), _ptr(out["delay"]),
                                   _ptr(out["slew"]), _ptr(tr.status), tr.stream()), "sta_tree_dataset")
    return out


def features(tr: Trees, feat=None):
    """Features [S][12] only (sta_tree_features: no moment sweeps)."""
    import torch
    if feat is None:
        feat = torch.empty((tr.n_sinks, 12), dtype=torch.float32, device=tr.device)
    _check(_lib().sta_tree_features(ctypes.byref(tr.c), _ptr(feat), _ptr(tr.status), tr.stream()),
           "sta_tree_features")
    return feat


def exact(tr: Trees, delay=None, slew=None, net_list=None, net_count=None):
    """Exact delay/slew per sink (all nets, or the listed ones)."""
    import torch
    if delay is None:
        delay = torch.empty(tr.n_sinks, dtype=torch.float32, device=tr.device)
    if slew is None:
        slew = torch.empty(tr.n_sinks, dtype=torch.float32, device=tr.device)
    _check(_lib().sta_tree_exact(ctypes.byref(tr.c), _ptr(net_list), _ptr(net_count), _ptr(delay), _ptr(slew),
                                 _ptr(tr.status), tr.stream()), "sta_tree_exact")
    return delay, slew


def norm_stats(feat):
    import torch
    lib = _lib()
    norm = torch.empty(24, dtype=torch.float32, device=feat.device)
    nb = lib.sta_mlp_norm_scratch_bytes()
    scratch = torch.empty(nb, dtype=torch.uint8, device=feat.device)
    _check(lib.sta_mlp_norm(_ptr(feat), int(feat.shape[0]), _ptr(norm), _ptr(scratch), nb,
                            _stream(torch, feat.device)), "sta_mlp_norm")
    return norm


class Model:
    """Parameters (FP32, natural layout), input normalization, Adam state, calibration."""

    def __init__(self, params, norm, device="cuda"):
        import torch
        self.device = torch.device(device)
        self.params = torch.as_tensor(np.asarray(params, np.float32) if not torch.is_tensor(params) else params,
                                      dtype=torch.float32).to(self.device).contiguous()
        self.norm = torch.as_tensor(norm, dtype=torch.float32).to(self.device).contiguous()
        self.m = torch.zeros(N_PARAMS, dtype=torch.float32, device=self.device)
        self.v = torch.zeros(N_PARAMS, dtype=torch.float32, device=self.device)
        self.step = 0
        self.calib = None

    @staticmethod
    def pack(p):
        """Flatten a dict of arrays (W1 [64][16] or [64][12], b1, W2, b2, W3, b3) into the vector."""
        v = np.zeros(N_PARAMS, np.float32)
        for k, (o, shp) in OFF.items():
            a = np.asarray(p[k], np.float32)
            if k == "W1" and a.shape == (64, 12):
                a = np.concatenate([a, np.zeros((64, 4), np.float32)], axis=1)
            v[o:o + int(np.prod(shp))] = a.reshape(-1)
        return v

    @staticmethod
    def unpack(v):
        v = np.asarray(v)
        return {k: v[o:o + int(np.prod(shp))].reshape(shp).copy() for k, (o, shp) in OFF.items()}

    def save(self, path):
        """Raw little-endian FP32 parameters and normalization (+ calibration) and JSON metadata."""
        base = os.path.splitext(path)[0]
        parts = [self.params.cpu().numpy(), self.norm.cpu().numpy()]
        if self.calib is not None:
            parts.append(self.calib.cpu().numpy().reshape(-1))
        np.concatenate(parts).astype("<f4").tofile(base + ".bin")
        meta = {"format": "sta-mlp-12-64-64-2", "params": N_PARAMS, "norm": 24,
                "calib": 0 if self.calib is None else CAL_BINS * 2, "offsets": {k: o for k, (o, _) in OFF.items()},
                "adam_step": self.step}
        with open(base + ".json", "w") as f:
            json.dump(meta, f, indent=1)

    @classmethod
    def load(cls, path, device="cuda"):
        import torch
        base = os.path.splitext(path)[0]
        with open(base + ".json") as f:
            meta = json.load(f)
        if meta.get("format") != "sta-mlp-12-64-64-2":
            raise ValueError("not a 12-64-64-2 surrogate checkpoint")
        raw = np.fromfile(base + ".bin", dtype="<f4")
        if raw.size != meta["params"] + meta["norm"] + meta["calib"]:
            raise ValueError("checkpoint size does not match its metadata")
        m = cls(raw[:N_PARAMS], raw[N_PARAMS:N_PARAMS + 24], device)
        if meta["calib"]:
            m.calib = torch.from_numpy(raw[N_PARAMS + 24:].reshape(CAL_BINS, 2).copy()).to(m.device)
        m.step = int(meta.get("adam_step", 0))
        return m


def train_step(model: Model, feat, target, idx, lr=None, betas=(0.9, 0.999), eps=1e-8, grad=None, scratch=None):
    """One forward/backward over feat[idx]; with lr, one Adam update.  Returns the gradient
    vector (N_PARAMS gradients + loss) if ``grad`` is given."""
    import torch
    lib = _lib()
    batch = int(idx.shape[0])
    nb = lib.sta_mlp_grad_scratch_bytes(batch)
    if scratch is None or scratch.numel() < nb:
        scratch = torch.empty(nb, dtype=torch.uint8, device=model.device)
    opt = None
    if lr is not None:
        model.step += 1
        opt = AdamC(float(lr), float(betas[0]), float(betas[1]), float(eps), model.step)
    _check(lib.sta_mlp_train_step(_ptr(model.params), _ptr(model.m), _ptr(model.v),
                                  ctypes.byref(opt) if opt is not None else None, _ptr(model.norm), _ptr(feat),
                                  _ptr(target), _ptr(idx), batch, _ptr(grad), _ptr(scratch), scratch.numel(),
                                  _stream(torch, model.device)), "sta_mlp_train_step")
    return grad


def predict(model: Model, feat, out=None):
    import torch
    n = int(feat.shape[0])
    if out is None:
        out = torch.empty((n, 2), dtype=torch.float32, device=model.device)
    _check(_lib().sta_mlp_predict(_ptr(model.params), _ptr(model.norm), _ptr(feat), n, _ptr(out),
                                  _stream(torch, model.device)), "sta_mlp_predict")
    return out


def calibrate(model: Model, feat, target, y, quantile=0.999, min_count=256):
    import torch
    lib = _lib()
    nb = lib.sta_surrogate_cal_scratch_bytes()
    scratch = torch.empty(nb, dtype=torch.uint8, device=model.device)
    calib = torch.empty((CAL_BINS, 2), dtype=torch.float32, device=model.device)
    _check(lib.sta_surrogate_calibrate(_ptr(feat), _ptr(target), _ptr(y), int(feat.shape[0]), float(quantile),
                                       int(min_count), _ptr(calib), _ptr(scratch), nb, _stream(torch, model.device)),
           "sta_surrogate_calibrate")
    model.calib = calib
    return calib


class EvalBuffers:
    def __init__(self, tr: Trees):
        import torch
        d = tr.device
        self.delay = torch.empty(tr.n_sinks, dtype=torch.float32, device=d)
        self.slew = torch.empty(tr.n_sinks, dtype=torch.float32, device=d)
        self.sink_flag = torch.empty(max(tr.n_sinks, 1), dtype=torch.uint8, device=d)
        self.flag = torch.empty(max(tr.n_nets, 1), dtype=torch.int32, device=d)
        self.list = torch.empty(max(tr.n_nets, 1), dtype=torch.int32, device=d)
        self.count = torch.zeros(1, dtype=torch.int32, device=d)


def evaluate(tr: Trees, model: Model, feat, tol_ps=1.0, buf: EvalBuffers = None):
    """The surrogate path: network + decode + error bound + exact fallback of untrusted nets."""
    if model.calib is None:
        raise ValueError("the model has no calibration")
    buf = buf or EvalBuffers(tr)
    _check(_lib().sta_surrogate_eval(ctypes.byref(tr.c), _ptr(model.params), _ptr(model.norm), _ptr(model.calib),
                                     _ptr(feat), float(tol_ps), _ptr(buf.delay), _ptr(buf.slew), _ptr(buf.sink_flag),
                                     _ptr(buf.flag),
                                     _ptr(buf.list), _ptr(buf.count), _ptr(tr.status), tr.stream()),
           "sta_surrogate_eval")
    return buf


def init_params(seed=0):
    """He-normal initialization (numpy, seeded), zero biases; W3 scaled by 0.5."""
    rng = np.random.default_rng(seed)
    W1 = np.zeros((64, 16))
    W1[:, :12] = rng.standard_normal((64, 12)) * math.sqrt(2.0 / 12)
    p = {"W1": W1, "b1": np.zeros(64), "W2": rng.standard_normal((64, 64)) * math.sqrt(2.0 / 64),
         "b2": np.zeros(64), "W3": rng.standard_normal((2, 64)) * math.sqrt(2.0 / 64) * 0.5, "b3": np.zeros(2)}
    return Model.pack(p)


def train(model: Model, feat, target, rows, steps, batch=8192, lr=2e-3, lr_min=2e-5, seed=0, log_every=0):
    """Adam over mini-batches drawn without replacement from ``rows`` (a permutation per
    epoch, seeded numpy), cosine learning-rate decay from lr to lr_min.  Returns the
    per-step losses (read back once at the end)."""
    import torch
    rng = np.random.default_rng(seed)
    rows = np.asarray(rows, np.int32)
    order = np.empty(0, np.int32)
    losses = torch.empty(steps, dtype=torch.float32, device=model.device)
    grad = torch.empty(N_PARAMS + 1, dtype=torch.float32, device=model.device)
    scratch = torch.empty(_lib().sta_mlp_grad_scratch_bytes(batch), dtype=torch.uint8, device=model.device)
    chunks = []
    need = steps * batch
    while sum(c.size for c in chunks) < need:
        chunks.append(rng.permutation(rows).astype(np.int32))
    order = np.concatenate(chunks)[:need]
    idx_all = torch.from_numpy(order).to(model.device)
    for k in range(steps):
        cur = lr_min + 0.5 * (lr - lr_min) * (1.0 + math.cos(math.pi * k / max(steps - 1, 1)))
        train_step(model, feat, target, idx_all[k * batch:(k + 1) * batch], lr=cur, grad=grad, scratch=scratch)
        losses[k:k + 1].copy_(grad[N_PARAMS:N_PARAMS + 1])
        if log_every and (k + 1) % log_every == 0:
            print(f"[train] step {k + 1}/{steps} loss {float(losses[k].item()):.3e}", flush=True)
    return losses.cpu().numpy()
