"""Python front end of the HIP renderer: workspace management, the four calls
of a frame, and a ``torch.autograd.Function``.

Only marshalling lives here: parameter tensors and views are turned into the
C structs of ``include/ubs.h``, device memory comes from torch, and every step
of the rendering runs in the HIP kernels of ``libubs.so``.
"""
from __future__ import annotations

import ctypes
import dataclasses
from typing import List, Optional, Sequence

import torch

from . import _lib
from ._lib import UbsFrame, UbsLayout, UbsScene, UbsTuning, UbsView

REC_FIELDS = ("mx", "my", "a", "b", "c", "rho", "o", "beta", "r", "g", "bl", "depth")


DEFAULT_TILE_SLOTS = 256   # slot block of a tile when tuning.tile_slots is 0
MAX_TILE_SLOTS = 4096


@dataclasses.dataclass
class Tuning:
    tile_w: int = 16
    tile_h: int = 16
    batch_depth: int = 64
    digit_bits: int = 8
    pair_capacity: int = 0          # 0: sized from the frame
    flags: int = 0
    tile_slots: int = 0             # 0: 256, grown by Renderer.forward after a spill

    def to_c(self, capacity: int) -> UbsTuning:
        return UbsTuning(self.tile_w, self.tile_h, self.batch_depth, self.digit_bits,
                         int(capacity), int(self.flags), int(self.tile_slots))


@dataclasses.dataclass
class SceneRef:
    """A scene for the renderer: float32 device tensor [F][n] plus format."""
    params: torch.Tensor
    dim: int
    rot: int = _lib.UBS_ROT_QUAT
    dparams: Optional[torch.Tensor] = None

    @property
    def n(self) -> int:
        return int(self.params.shape[1])


def _view_to_c(v) -> UbsView:
    R = [float(x) for x in torch.as_tensor(v.R, dtype=torch.float64).reshape(-1).tolist()]
    t = [float(x) for x in torch.as_tensor(v.t, dtype=torch.float64).reshape(-1).tolist()]
    c = UbsView()
    c.scene = int(getattr(v, "scene", 0))
    c.width = int(v.width)
    c.height = int(v.height)
    c.R = (ctypes.c_float * 9)(*R)
    c.t = (ctypes.c_float * 3)(*t)
    c.fx, c.fy, c.cx, c.cy = float(v.fx), float(v.fy), float(v.cx), float(v.cy)
    c.time = float(getattr(v, "time", 0.0))
    extra = [float(x) for x in getattr(v, "query", ())][:3]
    c.query = (ctypes.c_float * 3)(*(extra + [0.0] * (3 - len(extra))))
    return c


class FrameDesc:
    """Owns the ctypes arrays of one frame description."""

    def __init__(self, scenes: Sequence[SceneRef], views: Sequence, tuning: Tuning, capacity: int):
        self.scenes = list(scenes)
        self.views = list(views)
        self.tuning = tuning
        self._sc = (UbsScene * max(1, len(self.scenes)))()
        for k, s in enumerate(self.scenes):
            if s.params.dtype != torch.float32 or not s.params.is_contiguous():
                raise ValueError("scene params must be contiguous float32 [F][n]")
            self._sc[k] = UbsScene(int(s.dim), int(s.rot), s.n, s.params.data_ptr() if s.n else None,
                                   s.dparams.data_ptr() if s.dparams is not None and s.n else None)
        self._vw = (UbsView * max(1, len(self.views)))()
        for k, v in enumerate(self.views):
            self._vw[k] = _view_to_c(v)
        self.c = UbsFrame(self._sc, len(self.scenes), len(self.views), self._vw,
                          tuning.to_c(capacity))

    def set_dparams(self, k: int, t: Optional[torch.Tensor]) -> None:
        self.scenes[k].dparams = t
        self._sc[k].dparams = t.data_ptr() if t is not None and t.numel() else None

    def set_capacity(self, cap: int) -> None:
        self.c.tuning.pair_capacity = int(cap)

    def set_tile_slots(self, slots: int) -> None:
        self.c.tuning.tile_slots = int(slots)


def _stream() -> int:
    return torch.cuda.current_stream().cuda_stream


class Renderer:
    """Runs frames through the four C entry points on torch's current stream.

    The workspace is a torch uint8 tensor sized by the library's layout query;
    it grows when a frame needs more (tile, record) pairs than it holds.
    """

    def __init__(self, tuning: Optional[Tuning] = None, device: str = "cuda"):
        self.tuning = tuning or Tuning()
        self.device = torch.device(device)
        self.ws: Optional[torch.Tensor] = None
        self.layout: Optional[UbsLayout] = None
        self.frame: Optional[FrameDesc] = None
        self.capacity = int(self.tuning.pair_capacity)
        self.tile_slots = int(self.tuning.tile_slots)
        self.generation = 0

    # ---------------------------------------------------------------- layout
    def _plan(self, frame: FrameDesc) -> UbsLayout:
        lay = UbsLayout()
        _lib.ubs_preprocess(frame.c, 0, 0, lay, 0)
        return lay

    def _ensure_ws(self, frame: FrameDesc) -> None:
        lay = self._plan(frame)
        if self.ws is None or self.ws.numel() < lay.bytes:
            self.ws = torch.empty(max(int(lay.bytes), 256), dtype=torch.uint8, device=self.device)
            if self.ws.data_ptr() % 256:
                raise RuntimeError("workspace is not 256-byte aligned")
        self.layout = lay

    def make_frame(self, scenes: Sequence[SceneRef], views: Sequence) -> FrameDesc:
        n_rec = sum(scenes[int(getattr(v, "scene", 0))].n for v in views)
        if self.capacity <= 0:
            self.capacity = 2 * n_rec + (1 << 16)
        return FrameDesc(scenes, views, self.tuning, self.capacity)

    # ---------------------------------------------------------------- calls
    def preprocess(self, frame: FrameDesc) -> None:
        self._ensure_ws(frame)
        _lib.ubs_preprocess(frame.c, self.ws.data_ptr(), self.ws.numel(), self.layout, _stream())
        self.frame = frame
        self.generation += 1

    def bin_sort(self, frame: FrameDesc) -> None:
        _lib.ubs_bin_sort(frame.c, self.ws.data_ptr(), self.ws.numel(), _stream())

    def render_fwd(self, frame: FrameDesc, image: torch.Tensor, t_final: Optional[torch.Tensor]) -> None:
        _lib.ubs_render_fwd(frame.c, self.ws.data_ptr(), self.ws.numel(), image.data_ptr(),
                            t_final.data_ptr() if t_final is not None else 0, _stream())

    def render_bwd(self, frame: FrameDesc, d_image: Optional[torch.Tensor] = None,
                   d_t_final: Optional[torch.Tensor] = None, l1_image: Optional[torch.Tensor] = None,
                   l1_target: Optional[torch.Tensor] = None) -> None:
        ptr = lambda t: t.data_ptr() if t is not None else 0  # noqa: E731
        _lib.ubs_render_bwd(frame.c, self.ws.data_ptr(), self.ws.numel(), ptr(d_image),
                            ptr(d_t_final), ptr(l1_image), ptr(l1_target), _stream())

    # ---------------------------------------------------------------- helpers
    def status(self) -> dict:
        """Reads the status block (synchronises the stream)."""
        off = self.layout.off_status
        raw = self.ws[off:off + 64].cpu().numpy().tobytes()
        st = _lib.UbsStatusBlock.from_buffer_copy(raw)
        return {"pairs_needed": int(st.pairs_needed), "overflow": int(st.overflow),
                "n_nonfinite": int(st.n_nonfinite), "n_visible": int(st.n_visible),
                "sort_stalled": int(st.sort_stalled), "spill": int(st.spill)}

    def region(self, off: int, count: int, dtype: torch.dtype) -> torch.Tensor:
        esz = torch.tensor([], dtype=dtype).element_size()
        return self.ws[off:off + count * esz].view(dtype)

    def records(self) -> torch.Tensor:
        """The records in the workspace, [n_records][12] (a view: only the
        live ones are written by the preprocess, see ``record_live``)."""
        return self.region(self.layout.off_records, 12 * self.layout.n_records, torch.float32).view(-1, 12)

    def record_live(self) -> torch.Tensor:
        """Per record, 1 if it survived culling (uint8 view)."""
        return self.region(self.layout.off_live, self.layout.n_records, torch.uint8)

    def live_records(self) -> torch.Tensor:
        """A copy of the records with the culled ones zeroed."""
        rec = self.records()
        return torch.where(self.record_live().bool()[:, None], rec, torch.zeros((), dtype=rec.dtype,
                                                                                device=rec.device))

    def grad2d(self) -> torch.Tensor:
        return self.region(self.layout.off_grad2d, 10 * self.layout.n_records, torch.float32).view(-1, 10)

    def sorted_pairs(self, count: int):
        keys = self.region(self.layout.off_keys, count, torch.int64)
        vals = self.region(self.layout.off_values, count, torch.int32)
        return keys, vals

    def ranges(self) -> torch.Tensor:
        return self.region(self.layout.off_ranges, 2 * self.layout.n_tiles, torch.int32).view(-1, 2)

    def ncontrib(self) -> torch.Tensor:
        return self.region(self.layout.off_ncontrib, self.layout.n_pixels, torch.int32)

    # ---------------------------------------------------------------- frame
    def forward(self, scenes: Sequence[SceneRef], views: Sequence, *, check: bool = True):
        """preprocess -> bin_sort -> render_fwd.  Returns (image, t_final), each
        concatenated over views ([sum HW, 3] and [sum HW]).  With ``check``, reads
        the status once (one stream synchronisation) and reruns with a larger
        pair capacity if the frame overflowed; if a tile outgrew its slot block
        (a correct but slower frame) and the tuning leaves tile_slots to the
        renderer, the blocks are enlarged to fit the longest tile (up to 4096)
        and the frame is run again."""
        frame = self.make_frame(scenes, views)
        n_pix = sum(int(v.width) * int(v.height) for v in views)
        image = torch.empty((n_pix, 3), dtype=torch.float32, device=self.device)
        t_final = torch.empty((n_pix,), dtype=torch.float32, device=self.device)
        for _ in range(4):
            frame.set_capacity(self.capacity)
            frame.set_tile_slots(self.tile_slots)
            self.preprocess(frame)
            self.bin_sort(frame)
            if not check:
                break
            st = self.status()
            if st["overflow"]:
                self.capacity = int(st["pairs_needed"] * 1.25) + 1024
                continue
            if st["spill"] and self.tuning.tile_slots == 0:
                rg = self.ranges()
                longest = int((rg[:, 1] - rg[:, 0]).max().item())
                want = min(MAX_TILE_SLOTS, -(-int(longest * 1.25) // 64) * 64)
                if want > max(self.tile_slots, DEFAULT_TILE_SLOTS):
                    self.tile_slots = want
                    continue
            break
        self.render_fwd(frame, image, t_final)
        return image, t_final

    def backward(self, d_image: Optional[torch.Tensor] = None, d_t_final: Optional[torch.Tensor] = None,
                 *, l1_image: Optional[torch.Tensor] = None, l1_target: Optional[torch.Tensor] = None):
        """render_bwd of the last frame; returns dparams per scene."""
        frame = self.frame
        outs = []
        for k, s in enumerate(frame.scenes):
            g = torch.empty_like(s.params)
            frame.set_dparams(k, g)
            outs.append(g)
        self.render_bwd(frame, d_image, d_t_final, l1_image, l1_target)
        return outs


def split_views(flat: torch.Tensor, views: Sequence) -> List[torch.Tensor]:
    """Splits a [sum HW, ...] tensor into per-view [H, W, ...] tensors."""
    out, k = [], 0
    for v in views:
        n = int(v.width) * int(v.height)
        out.append(flat[k:k + n].view(int(v.height), int(v.width), *flat.shape[1:]))
        k += n
    return out


class UBSRenderFunction(torch.autograd.Function):
    """image, t_final = f(params_0, ..., params_{S-1}); backward is the
    hand-written adjoint of ``ubs_render_bwd``."""

    @staticmethod
    def forward(ctx, renderer: Renderer, dims: tuple, rots: tuple, views: tuple, *params):
        scenes = [SceneRef(p.detach(), d, r) for p, d, r in zip(params, dims, rots)]
        image, t_final = renderer.forward(scenes, list(views))
        ctx.renderer = renderer
        ctx.generation = renderer.generation
        # an output the loss does not use arrives in backward as None (no
        # zero tensor, so no transmittance term is read for it)
        ctx.set_materialize_grads(False)
        return image, t_final

    @staticmethod
    def backward(ctx, d_image, d_t_final):
        r = ctx.renderer
        if r.generation != ctx.generation:
            raise RuntimeError("the renderer ran another frame before this backward")
        if d_image is None and d_t_final is None:
            return (None, None, None, None) + (None,) * len(r.frame.scenes)
        if d_image is None:   # the C call takes d_image whenever d_t_final is given
            d_image = torch.zeros((r.layout.n_pixels, 3), dtype=torch.float32, device=r.device)
        d_image = d_image.to(torch.float32).contiguous()
        if d_t_final is not None:
            d_t_final = d_t_final.to(torch.float32).contiguous()
        grads = r.backward(d_image, d_t_final)
        return (None, None, None, None, *grads)


def render(renderer: Renderer, params: Sequence[torch.Tensor], dims: Sequence[int],
           rots: Sequence[int], views: Sequence):
    """Differentiable render of every view; returns (image, t_final) flat over views."""
    return UBSRenderFunction.apply(renderer, tuple(dims), tuple(rots), tuple(views), *params)


class GraphFrame:
    """One forward+backward frame captured in a HIP graph and replayed.

    The frame is first run eagerly (sizing the workspace and the pair
    capacity), then the four calls are captured with ``torch.cuda.graph``.
    Every replay re-renders from the current contents of the parameter
    tensors and writes ``image``, ``t_final`` and the ``dparams`` tensors.
    The pair capacity is fixed at capture: after a replay, ``status()``
    reports ``overflow`` if a frame needed more (re-create the GraphFrame).
    Loss: ``l1_target`` (fused L1 gradient) or ``d_image`` (a tensor whose
    contents are read at each replay).
    """

    def __init__(self, renderer: Renderer, scenes: Sequence[SceneRef], views: Sequence, *,
                 l1_target: Optional[torch.Tensor] = None, d_image: Optional[torch.Tensor] = None,
                 backward: bool = True, headroom: float = 1.25):
        if backward and (l1_target is None) == (d_image is None):
            raise ValueError("give exactly one of l1_target or d_image")
        self.r = renderer
        self.views = list(views)
        self.l1_target, self.d_image = l1_target, d_image
        self.image, self.t_final = renderer.forward(scenes, self.views)   # sizes the capacity
        st = renderer.status()
        cap = max(renderer.capacity, int(st["pairs_needed"] * headroom) + 1024)
        if cap != renderer.capacity:
            renderer.capacity = cap
            self.image, self.t_final = renderer.forward(scenes, self.views)
        self.frame = renderer.frame
        self.dparams = []
        for k, s in enumerate(self.frame.scenes):
            g = torch.empty_like(s.params)
            self.frame.set_dparams(k, g)
            self.dparams.append(g)
        self.backward = backward
        self._step()                       # eager warm-up of the exact sequence
        torch.cuda.synchronize()
        self.graph = self.capture()

    def capture(self) -> "torch.cuda.CUDAGraph":
        """Captures the frame once more into a new graph (per-stage timing is
        taken from plain calls, ``step()`` with a ``StageTimer`` attached)."""
        g = torch.cuda.CUDAGraph()
        self.frame.c.stage_events = None
        with torch.cuda.graph(g):
            self._step()
        torch.cuda.synchronize()
        return g

    def step(self) -> None:
        """Runs the frame eagerly (the sequence the graphs replay)."""
        self._step()

    def _step(self) -> None:
        r, f = self.r, self.frame
        r.preprocess(f)
        r.bin_sort(f)
        r.render_fwd(f, self.image, self.t_final)
        if self.backward:
            if self.l1_target is not None:
                r.render_bwd(f, l1_image=self.image, l1_target=self.l1_target)
            else:
                r.render_bwd(f, self.d_image)

    def replay(self) -> None:
        self.graph.replay()

    def status(self) -> dict:
        return self.r.status()
