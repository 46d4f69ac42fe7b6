"""The learned warm start's network on the device: parameters, inference,
statistics, gradients, Adam, and the logger that turns solved steps into
training rows.  Argument marshalling over the C ABI; the arithmetic runs in
the HIP library.

    net = Net(device="cuda:0", seed=0)
    x, t = gather(sim)                  # after a tight step with export on
    net.fit_stats(x)
    loss = net.train_step(x, t, rows, lr=1e-4)
    net.attach(sim)                     # the step then runs it in LEARNED mode
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _lib as L

NP, NW, NB = L.MLP_NPARAM, L.MLP_NWEIGHT, L.MLP_NBIAS
# flat fp32 parameter order: w1 [64][16] | b1 [64] | w2 [64][64] | b2 [64] | w3 [3][64] | b3 [3]
SLICES = {"w1": (0, 1024, (64, 16)), "b1": (1024, 1088, (64,)), "w2": (1088, 5184, (64, 64)),
          "b2": (5184, 5248, (64,)), "w3": (5248, 5440, (3, 64)), "b3": (5440, 5443, (3,))}


def _p(t: torch.Tensor | None):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def _stream(device: torch.device):
    return C.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def init_params(seed: int = 0) -> np.ndarray:
    """He-uniform weights for the ReLU layers, zero biases (host, float32)."""
    rng = np.random.default_rng(seed)
    out = np.zeros(NP, np.float32)
    for name, fan_in in (("w1", 16), ("w2", 64), ("w3", 64)):
        a, b, shape = SLICES[name]
        lim = np.sqrt(6.0 / fan_in) if name != "w3" else np.sqrt(3.0 / fan_in)
        out[a:b] = rng.uniform(-lim, lim, size=b - a).astype(np.float32)
    return out


def unflatten(flat) -> dict:
    """Split a flat parameter vector into named arrays (float64, host)."""
    flat = np.asarray(flat, np.float64)
    return {k: flat[a:b].reshape(s) for k, (a, b, s) in SLICES.items()}


class Net:
    """Master parameters, Adam moments and the bf16 inference copy, all on one device."""

    def __init__(self, device: str | torch.device = "cuda", seed: int = 0, params: np.ndarray | None = None):
        self.lib = L.load()
        self.device = torch.device(device)
        if self.device.type == "cuda" and self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        p = init_params(seed) if params is None else np.asarray(params, np.float32)
        if p.shape != (NP,):
            raise ValueError(f"params must hold {NP} values")
        f32 = dict(dtype=torch.float32, device=self.device)
        self.params = torch.tensor(p, **f32)
        self.m = torch.zeros(NP, **f32)
        self.v = torch.zeros(NP, **f32)
        self.grad = torch.zeros(NP, **f32)
        self.loss = torch.zeros(1, **f32)
        self.gnorm = torch.zeros(1, **f32)
        self.mean = torch.zeros(16, **f32)
        self.std = torch.ones(16, **f32)
        self.wbf = torch.zeros(NW, dtype=torch.bfloat16, device=self.device)
        self.bias = torch.zeros(NB, **f32)
        self.step_count = 0
        self._work = torch.zeros(0, dtype=torch.uint8, device=self.device)
        self.export()

    # ---------------------------------------------------------------- helpers
    def _workspace(self, n: int) -> torch.Tensor:
        need = int(self.lib.sim_mlp_workspace_bytes(int(n)))
        if self._work.numel() < need:
            self._work = torch.zeros(need + 256, dtype=torch.uint8, device=self.device)
        return self._work

    def _check_rows(self, x: torch.Tensor, width: int, name: str):
        if x.device != self.device or x.dtype != torch.float32 or not x.is_contiguous() or x.dim() != 2 \
                or x.shape[1] != width:
            raise ValueError(f"{name} must be a contiguous float32 [n, {width}] tensor on {self.device}")

    def weights(self) -> L.MlpWeights:
        """Inference pointers (bf16 w1 | w2 | w3 and b1 | b2 | b3, plus mean and std)."""
        wb, bs = self.wbf.data_ptr(), self.bias.data_ptr()
        return L.MlpWeights(wb, wb + 2 * 1024, wb + 2 * 5120, bs, bs + 4 * 64, bs + 4 * 128,
                            self.mean.data_ptr(), self.std.data_ptr())

    def named(self) -> dict:
        """Named float64 host copies of the master parameters plus mean and std."""
        d = unflatten(self.params.cpu().numpy())
        d["mean"] = self.mean.cpu().numpy().astype(np.float64)
        d["std"] = self.std.cpu().numpy().astype(np.float64)
        return d

    # ---------------------------------------------------------------- kernels
    def export(self):
        """Refresh the bf16 inference copy from the master parameters."""
        L.check(self.lib.sim_mlp_export(_p(self.params), _p(self.wbf), _p(self.bias), _stream(self.device)),
                "sim_mlp_export")

    def fit_stats(self, x: torch.Tensor):
        """Feature mean and std of a training set x [n, 16]."""
        self._check_rows(x, 16, "x")
        w = self._workspace(x.shape[0])
        L.check(self.lib.sim_mlp_stats(_p(x), int(x.shape[0]), _p(self.mean), _p(self.std), _p(w), w.numel(),
                                       _stream(self.device)), "sim_mlp_stats")

    def forward(self, x: torch.Tensor) -> torch.Tensor:
        self._check_rows(x, 16, "x")
        y = torch.empty((x.shape[0], 3), dtype=torch.float32, device=self.device)
        w = self.weights()
        L.check(self.lib.sim_mlp_forward(C.byref(w), _p(x), int(x.shape[0]), _p(y), _stream(self.device)),
                "sim_mlp_forward")
        return y

    def compute_grad(self, x: torch.Tensor, t: torch.Tensor, rows: torch.Tensor | None = None,
                     n: int | None = None) -> torch.Tensor:
        """Gradient of the batch loss into self.grad (and the loss into self.loss)."""
        self._check_rows(x, 16, "x")
        self._check_rows(t, 3, "t")
        if rows is not None:
            if rows.dtype != torch.int32 or rows.device != self.device or not rows.is_contiguous():
                raise ValueError("rows must be a contiguous int32 device tensor")
            n = int(rows.numel()) if n is None else int(n)
        else:
            n = int(x.shape[0]) if n is None else int(n)
        w = self._workspace(n)
        L.check(self.lib.sim_mlp_grad(_p(self.params), _p(self.mean), _p(self.std), _p(x), _p(t), _p(rows), n,
                                      _p(self.grad), _p(self.loss), _p(w), w.numel(), _stream(self.device)),
                "sim_mlp_grad")
        return self.grad

    def compute_grad_noalloc(self, x: torch.Tensor, t: torch.Tensor, rows: torch.Tensor | None = None,
                             n: int | None = None) -> torch.Tensor:
        """compute_grad through sim_mlp_grad_noalloc: no workspace, at most
        sim_mlp_grad_noalloc_max_rows() rows."""
        self._check_rows(x, 16, "x")
        self._check_rows(t, 3, "t")
        if rows is not None:
            if rows.dtype != torch.int32 or rows.device != self.device or not rows.is_contiguous():
                raise ValueError("rows must be a contiguous int32 device tensor")
            n = int(rows.numel()) if n is None else int(n)
        else:
            n = int(x.shape[0]) if n is None else int(n)
        L.check(self.lib.sim_mlp_grad_noalloc(_p(self.params), _p(self.mean), _p(self.std), _p(x), _p(t), _p(rows),
                                              n, _p(self.grad), _p(self.loss), _stream(self.device)),
                "sim_mlp_grad_noalloc")
        return self.grad

    def adam(self, lr: float, clip: float = 0.5):
        self.step_count += 1
        L.check(self.lib.sim_mlp_adam(_p(self.params), _p(self.m), _p(self.v), _p(self.grad), self.step_count,
                                      float(lr), float(clip), _p(self.gnorm), _stream(self.device)), "sim_mlp_adam")

    def train_step(self, x, t, rows=None, lr: float = 1e-4, clip: float = 0.5):
        self.compute_grad(x, t, rows)
        self.adam(lr, clip)
        return self.loss

    def attach(self, sim):
        """Use this network for the learned warm start of sim (keeps the buffers alive)."""
        self.export()
        w = self.weights()
        sim._mlp = self
        L.check(self.lib.sim_set_mlp(sim.h, w.w1, w.w2, w.w3, w.b1, w.b2, w.b3, w.mean, w.std), "sim_set_mlp")


def gather(sim, cap: int | None = None, target_clip: float = 0.0):
    """Training rows (features [n, 16], scaled targets [n, 3], saturated at
    +-target_clip when > 0) of the sim's last step."""
    lib = L.load()
    cap = int(cap if cap is not None else sim.S * sim.max_contacts)
    x = torch.empty((max(cap, 1), 16), dtype=torch.float32, device=sim.device)
    t = torch.empty((max(cap, 1), 3), dtype=torch.float32, device=sim.device)
    total = torch.zeros(1, dtype=torch.int64, device=sim.device)
    L.check(lib.sim_mlp_gather(sim.h, _p(x), _p(t), cap, float(target_clip), _p(total)), "sim_mlp_gather")
    n = min(int(total.item()), cap)
    return x[:n], t[:n]


def train(net: Net, x: torch.Tensor, t: torch.Tensor, epochs: int = 10, batch: int = 4096, lr: float = 1e-4,
          clip: float = 0.5, seed: int = 0, log=None):
    """Minibatch Adam over (x, t) with the learning rate decayed linearly to 0."""
    n = int(x.shape[0])
    if n < 1:
        raise ValueError("empty training set")
    per_epoch = (n + batch - 1) // batch
    total = epochs * per_epoch
    g = torch.Generator(device=net.device)
    g.manual_seed(seed)
    k = 0
    for ep in range(epochs):
        perm = torch.randperm(n, generator=g, device=net.device).to(torch.int32)
        for b in range(per_epoch):
            rows = perm[b * batch:(b + 1) * batch]
            net.train_step(x, t, rows, lr=lr * (1.0 - k / total), clip=clip)
            k += 1
        if log is not None:
            log(ep, float(net.loss.item()))
    net.export()
    return net
