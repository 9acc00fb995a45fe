"""ctypes binding of the learned-correction C ABI (``include/ii_learned.h``).

Argument marshalling only: every step runs in the library's kernels; torch
tensors provide the device memory and the stream.  BF16 patches are held in
``torch.bfloat16`` tensors (the same bits the kernels read).
"""
from __future__ import annotations

import ctypes as C
from typing import Optional

import numpy as np

from . import binding as B

NPARAM = 22281
PATCH = 24
TILE = 16
CHANNELS = (4, 32, 32, 32, 9)
# parameter layout: W1 b1 W2 b2 W3 b3 W4 b4, W[dy][dx][ci][co]
_SHAPES = [(3, 3, 4, 32), (32,), (3, 3, 32, 32), (32,), (3, 3, 32, 32), (32,), (3, 3, 32, 9), (9,)]

EXPORTS = ["ii_cnn_packed_bytes", "ii_cnn_pack", "ii_cnn_save_bytes", "ii_cnn_forward",
           "ii_cnn_work_bytes", "ii_cnn_backward", "ii_cnn_adam", "ii_lbm_learned_tiles",
           "ii_lbm_learned_patches", "ii_lbm_learned_targets", "ii_lbm_learned_apply",
           "ii_lbm_learned_correct", "ii_lbm_learned_infer", "ii_lbm_set_learned"]


class Scales(C.Structure):
    _fields_ = [("in_scale", C.c_float * 4), ("out_scale", C.c_float)]


def make_scales(in_scale, out_scale) -> Scales:
    s = Scales()
    for c in range(4):
        s.in_scale[c] = float(in_scale[c])
    s.out_scale = float(out_scale)
    return s


_reg = False


def lib():
    global _reg
    L = B.load()
    if not _reg:
        v, i32, sz = C.c_void_p, C.c_int32, C.c_size_t
        S = C.POINTER(Scales)
        sig = {
            "ii_cnn_packed_bytes": ([], sz), "ii_cnn_save_bytes": ([], sz),
            "ii_cnn_work_bytes": ([i32], sz),
            "ii_cnn_pack": ([v, v, v], C.c_int),
            "ii_cnn_forward": ([v, v, v, i32, v, v, v], C.c_int),
            "ii_cnn_backward": ([v, v, v, v, v, v, v, i32, v, v, v, v], C.c_int),
            "ii_cnn_adam": ([v, v, v, v, i32, C.c_float, v, v], C.c_int),
            "ii_lbm_learned_tiles": ([v, i32, v, v], C.c_int),
            "ii_lbm_learned_patches": ([v, S, i32, v, v, v, v, v], C.c_int),
            "ii_lbm_learned_targets": ([v, v, S, i32, v, v, v, v, v, v], C.c_int),
            "ii_lbm_learned_apply": ([v, S, i32, v, v, v, v, v], C.c_int),
            "ii_lbm_learned_correct": ([v, v, v, S, i32, v, v, v, v, v], C.c_int),
            "ii_lbm_learned_infer": ([v, v, v, S, i32, v, v, v, v, v], C.c_int),
            "ii_lbm_set_learned": ([v, v, v, S, i32, v, v, v, v, v], C.c_int),
        }
        for name, (args, res) in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _reg = True
    return L


def _p(t) -> C.c_void_p:
    return C.c_void_p(0 if t is None else t.data_ptr())


def flatten_params(W, b) -> np.ndarray:
    """FP32 parameter vector from per-layer W[dy, dx, ci, co] and b[co]."""
    parts = []
    for l in range(4):
        parts += [np.asarray(W[l], dtype=np.float64).ravel(), np.asarray(b[l], dtype=np.float64).ravel()]
    out = np.concatenate(parts).astype(np.float32)
    assert out.size == NPARAM
    return out


def split_params(p: np.ndarray):
    """Per-layer (W, b) views of a parameter vector."""
    W, b, o = [], [], 0
    for k, s in enumerate(_SHAPES):
        n = int(np.prod(s))
        (W if k % 2 == 0 else b).append(np.asarray(p[o:o + n], dtype=np.float64).reshape(s))
        o += n
    return W, b


class Net:
    """FP32 master parameters, Adam moments and the packed BF16 fragments,
    all resident on the device."""

    def __init__(self, params: np.ndarray, device: str = "cuda:0", stream=None):
        import torch
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.params = torch.tensor(np.asarray(params, dtype=np.float32), device=self.device)
        assert self.params.numel() == NPARAM
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.t = 0
        self.packed = torch.empty(lib().ii_cnn_packed_bytes(), dtype=torch.uint8, device=self.device)
        self.pack()

    def _s(self):
        return C.c_void_p(self.stream.cuda_stream)

    def pack(self) -> None:
        B.check(lib().ii_cnn_pack(_p(self.params), _p(self.packed), self._s()), "ii_cnn_pack")

    def forward(self, inp, save: bool = False):
        """inp: bfloat16 [n, 24, 24, 4] -> (out float32 [n, 16, 16, 9], saved or None)."""
        import torch
        n = inp.shape[0]
        out = torch.empty((n, TILE, TILE, 9), dtype=torch.float32, device=self.device)
        sv = None
        if save:
            sv = torch.empty((n, lib().ii_cnn_save_bytes() // 2), dtype=torch.bfloat16, device=self.device)
        B.check(lib().ii_cnn_forward(_p(self.params), _p(self.packed), _p(inp), n, _p(out), _p(sv),
                                     self._s()), "ii_cnn_forward")
        return out, sv

    def backward(self, inp, saved, out, target, mask):
        """Gradient of the masked MSE and the loss (device tensors)."""
        import torch
        n = inp.shape[0]
        grad = torch.empty(NPARAM, dtype=torch.float32, device=self.device)
        loss = torch.empty(1, dtype=torch.float32, device=self.device)
        work = torch.empty(lib().ii_cnn_work_bytes(n), dtype=torch.uint8, device=self.device)
        B.check(lib().ii_cnn_backward(_p(self.params), _p(self.packed), _p(inp), _p(saved), _p(out),
                                      _p(target), _p(mask), n, _p(grad), _p(loss), _p(work),
                                      self._s()), "ii_cnn_backward")
        return grad, loss

    def adam(self, grad, lr: float = 1e-3) -> None:
        self.t += 1
        B.check(lib().ii_cnn_adam(_p(self.params), _p(grad), _p(self.m), _p(self.v), self.t, float(lr),
                                  _p(self.packed), self._s()), "ii_cnn_adam")

    def numpy(self) -> np.ndarray:
        return self.params.detach().cpu().numpy()


class Band:
    """Device scratch for the band tiles and patches of every instance of a
    handle (n_inst * cap slots)."""

    def __init__(self, sim: "B.Sim", cap: Optional[int] = None):
        import torch
        self.sim = sim
        tiles_per = [(p.nx // TILE) * (p.ny // TILE) for p in sim.problems]
        self.cap = int(cap if cap is not None else max(tiles_per))
        n = sim.n_inst * self.cap
        dev = sim.device
        self.tiles = torch.zeros(2 * n, dtype=torch.int32, device=dev)
        self.count = torch.zeros(sim.n_inst, dtype=torch.int32, device=dev)
        self.inp = torch.zeros((n, PATCH, PATCH, 4), dtype=torch.bfloat16, device=dev)
        self.flags = torch.zeros((n, PATCH, PATCH), dtype=torch.uint8, device=dev)
        self.pscale = torch.ones(n, dtype=torch.float32, device=dev)

    def find(self) -> None:
        B.check(lib().ii_lbm_learned_tiles(self.sim.h, self.cap, _p(self.tiles), _p(self.count)),
                "ii_lbm_learned_tiles")

    def patches(self, sc: Scales) -> None:
        B.check(lib().ii_lbm_learned_patches(self.sim.h, C.byref(sc), self.cap, _p(self.tiles),
                                             _p(self.count), _p(self.inp), _p(self.flags),
                                             _p(self.pscale)), "ii_lbm_learned_patches")

    def targets(self, fine: "B.Sim", sc: Scales):
        """(target float32 [n, 16, 16, 9], mask uint8 [n, 16, 16]) of the slots."""
        import torch
        n = self.sim.n_inst * self.cap
        tg = torch.zeros((n, TILE, TILE, 9), dtype=torch.float32, device=self.sim.device)
        mk = torch.zeros((n, TILE, TILE), dtype=torch.uint8, device=self.sim.device)
        B.check(lib().ii_lbm_learned_targets(self.sim.h, fine.h, C.byref(sc), self.cap, _p(self.tiles),
                                             _p(self.count), _p(self.flags), _p(self.pscale), _p(tg),
                                             _p(mk)), "ii_lbm_learned_targets")
        return tg, mk

    def apply(self, out, sc: Scales) -> None:
        """Masked add of given corrections (network units) to the listed tiles."""
        B.check(lib().ii_lbm_learned_apply(self.sim.h, C.byref(sc), self.cap, _p(self.tiles),
                                           _p(self.count), _p(self.flags), _p(self.pscale), _p(out)),
                "ii_lbm_learned_apply")

    def correct(self, net: Net, sc: Scales) -> None:
        B.check(lib().ii_lbm_learned_correct(self.sim.h, _p(net.params), _p(net.packed), C.byref(sc),
                                             self.cap, _p(self.tiles), _p(self.count), _p(self.inp),
                                             _p(self.flags), _p(self.pscale)), "ii_lbm_learned_correct")

    def infer(self, net: Net, sc: Scales) -> None:
        """The network and the masked add on the patches of the last `patches`."""
        B.check(lib().ii_lbm_learned_infer(self.sim.h, _p(net.params), _p(net.packed), C.byref(sc),
                                           self.cap, _p(self.tiles), _p(self.count), _p(self.inp),
                                           _p(self.flags), _p(self.pscale)), "ii_lbm_learned_infer")

    def attach(self, net: Net, sc: Scales) -> None:
        """Have the handle apply the correction after every step (its own
        stream schedule and graphs); the band scratch is this object's."""
        self._attached = (net, sc)   # the handle keeps pointers into both
        B.check(lib().ii_lbm_set_learned(self.sim.h, _p(net.params), _p(net.packed), C.byref(sc),
                                         self.cap, _p(self.tiles), _p(self.count), _p(self.inp),
                                         _p(self.flags), _p(self.pscale)), "ii_lbm_set_learned")

    def detach(self) -> None:
        B.check(lib().ii_lbm_set_learned(self.sim.h, None, None, None, 0, None, None, None, None,
                                         None), "ii_lbm_set_learned")
        self._attached = None

    def slots(self):
        """Indices of the filled slots (host)."""
        cnt = self.count.cpu().numpy()
        return np.concatenate([j * self.cap + np.arange(int(c)) for j, c in enumerate(cnt)]).astype(np.int64) \
            if cnt.sum() else np.zeros(0, np.int64)

    def tile_of(self, slot: int):
        t = self.tiles.view(-1, 2)[slot].cpu().numpy()
        return int(t[0]), int(t[1])
