"""MI355X-native Epstein-Nesbet MRPT2 energy in the STP-DAS organisation.

Python front end of libmrpt2.so.  PyTorch supplies device memory and the
stream; every step of the energy runs in the library's HIP kernels.  The
package fails loudly when the library is missing or no GPU is present: there
is no CPU fallback.
"""
import ctypes

import numpy as np

from . import capi
from .capi import CLASSES, Mrpt2Error  # noqa: F401


def make_desc(n_frozen_core, n_core, n_virt, sub_sizes, sub_base, max_hops, n_act_elec,
              sets, q_mode=0, precision=0, level_shift_b=0.0, layout=0):
    """Fill a descriptor.  sets = [(rank, weight), ...]; layout 0 passes
    each factor matrix in full [n][n], 1 as its packed upper triangle
    [n (n + 1) / 2] (see hermitian_pack)."""
    d = capi.Desc()
    d.n_frozen_core = n_frozen_core
    d.n_core = n_core
    d.n_virt = n_virt
    d.n_sub = len(sub_sizes)
    for k, (s, b) in enumerate(zip(sub_sizes, sub_base)):
        d.sub_size[k] = s
        d.sub_base[k] = b
    d.max_hops = max_hops
    d.n_act_elec = n_act_elec
    d.q_mode = q_mode
    d.n_sets = len(sets)
    for t, (r, w) in enumerate(sets):
        d.rank[t] = r
        d.weight[t] = w
    d.precision = precision
    d.level_shift_b = level_shift_b
    d.layout = layout
    return d


def desc_of_problem(pb, precision=0, q_mode=None, level_shift_b=0.0, layout=0):
    """Descriptor of a synth.problems.Problem."""
    return make_desc(pb.n_fc, pb.n_c, pb.n_v, pb.sub_sizes, pb.base, min(pb.max_hops, 1 << 20),
                     pb.n_elec, pb.sets, pb.q_mode if q_mode is None else q_mode, precision,
                     level_shift_b, layout)


def hermitian_pack(B):
    """Packed layout of Hermitian factor matrices: B [..., n, n] ->
    [..., n (n + 1) / 2], the upper triangle of each matrix by rows (entry
    (p, q), p <= q, at p n - p (p - 1) / 2 + (q - p)).  A copy in the
    caller's tensor library; the library reads the packed tensor directly."""
    import torch
    n = B.shape[-1]
    iu = torch.triu_indices(n, n, device=B.device)
    return B[..., iu[0], iu[1]].contiguous()


class Plan:
    """Host plan of one or more instances (no device work).  tuning: None
    (built-in launch shapes) or one capi.Tuning per instance (see autotune)."""

    def __init__(self, descs, tuning=None):
        if isinstance(descs, capi.Desc):
            descs = [descs]
        self.n_inst = len(descs)
        arr = (capi.Desc * self.n_inst)(*descs)
        self._descs = arr
        h = ctypes.c_void_p()
        if tuning is None:
            capi.check(capi.lib().mrpt2_plan(arr, self.n_inst, ctypes.byref(h)), "mrpt2_plan")
        else:
            if isinstance(tuning, capi.Tuning):
                tuning = [tuning]
            if len(tuning) != self.n_inst:
                raise ValueError("one Tuning per instance expected")
            tarr = (capi.Tuning * self.n_inst)(*tuning)
            capi.check(capi.lib().mrpt2_plan_tuned(arr, self.n_inst, tarr, ctypes.byref(h)), "mrpt2_plan_tuned")
        self.handle = h
        p, w = ctypes.c_size_t(), ctypes.c_size_t()
        capi.check(capi.lib().mrpt2_plan_sizes(h, ctypes.byref(p), ctypes.byref(w)), "mrpt2_plan_sizes")
        self.persistent_bytes = p.value
        self.workspace_bytes = w.value
        g = ctypes.c_size_t()
        capi.check(capi.lib().mrpt2_plan_backward_size(h, ctypes.byref(g)), "mrpt2_plan_backward_size")
        self.grad_bytes = g.value

    def info(self, inst=0):
        inf = capi.Info()
        capi.check(capi.lib().mrpt2_plan_info(self.handle, inst, ctypes.byref(inf)), "mrpt2_plan_info")
        return inf

    def ref_strings(self, inst=0):
        n = self.info(inst).n_ref
        out = np.zeros(n, dtype=np.uint64)
        capi.check(capi.lib().mrpt2_plan_ref_strings(
            self.handle, inst, out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))), "mrpt2_plan_ref_strings")
        return out

    def class_blocks(self, cls, inst=0):
        """Block descriptions (capi.Block) of class cls's partial sums."""
        n = ctypes.c_int64()
        capi.check(capi.lib().mrpt2_plan_class_blocks(self.handle, inst, cls, ctypes.byref(n)),
                   "mrpt2_plan_class_blocks")
        return n.value

    def class_block(self, cls, b, inst=0):
        out = capi.Block()
        capi.check(capi.lib().mrpt2_plan_class_block(self.handle, inst, cls, b, ctypes.byref(out)),
                   "mrpt2_plan_class_block")
        return out

    def class_strings(self, cls, inst=0):
        n = self.info(inst).n_strings_class[cls]
        out = np.zeros(max(n, 1), dtype=np.uint64)
        capi.check(capi.lib().mrpt2_plan_class_strings(
            self.handle, inst, cls, out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))), "mrpt2_plan_class_strings")
        return out[:n]

    def __del__(self):
        h = getattr(self, "handle", None)
        try:
            if h is not None and h.value:
                capi.lib().mrpt2_plan_destroy(h)
        except Exception:      # interpreter shutdown
            pass
        self.handle = None


def _require_gpu():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("paper_2608_11529_amd needs a ROCm GPU (gfx950); none is visible")
    return torch


class Engine:
    """A plan with its device regions, bound to one GPU and stream."""

    def __init__(self, plan, device="cuda:0", stream=None):
        torch = _require_gpu()
        self.torch = torch
        self.plan = plan
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.persistent = torch.empty(max(plan.persistent_bytes, 256), dtype=torch.uint8, device=self.device)
        self.workspace = torch.empty(max(plan.workspace_bytes, 256), dtype=torch.uint8, device=self.device)
        capi.check(capi.lib().mrpt2_plan_upload(plan.handle, self.persistent.data_ptr(), plan.persistent_bytes,
                                               self._sptr()), "mrpt2_plan_upload")
        self.e2 = torch.zeros(plan.n_inst, dtype=torch.float64, device=self.device)
        self.parts = torch.zeros((plan.n_inst, 12), dtype=torch.float64, device=self.device)

    def _sptr(self):
        return ctypes.c_void_p(self.stream.cuda_stream)

    def _inputs(self, insts, inst=None):
        """ctypes input sets: one per instance, or (inst given) the single set
        of instance inst."""
        if inst is None and len(insts) != self.plan.n_inst:
            raise ValueError("the plan holds %d instances, %d input sets given" % (self.plan.n_inst, len(insts)))
        if inst is not None and (len(insts) != 1 or not 0 <= inst < self.plan.n_inst):
            raise ValueError("one input set of an instance of the plan expected")
        arr = (capi.Inputs * len(insts))()
        keep = []
        for i, (h, Bs, c) in enumerate(insts):
            self._check_shapes(i if inst is None else inst, h, Bs, c)
            for x in [h, c, *Bs]:
                if x is not None:
                    if not x.is_contiguous() or x.device != self.device:
                        raise ValueError("inputs must be contiguous tensors on the engine's device")
                    keep.append(x)
            arr[i].h = h.data_ptr()
            for t, B in enumerate(Bs):
                arr[i].B[t] = B.data_ptr()
            arr[i].c = c.data_ptr() if c is not None else None
        return arr, keep

    def _check_shapes(self, i, h, Bs, c):
        """The kernels read exactly the sizes the plan fixes: h [n][n], B_t
        [rank_t][n][n], c [N_P] (or [n_roots][N_P]); anything else is refused
        here, before a device read could run past a tensor."""
        info, desc = self.plan.info(i), self.plan._descs[i]
        n = info.n_orb
        torch = self.torch
        if h is None or tuple(h.shape) != (n, n) or h.dtype != torch.complex128:
            raise ValueError("instance %d: h must be complex128 [%d, %d]" % (i, n, n))
        ranks = [desc.rank[t] for t in range(desc.n_sets)]
        if len(Bs) != len(ranks):
            raise ValueError("instance %d: %d factor sets expected" % (i, len(ranks)))
        packed = desc.layout == 1
        for t, (B, r) in enumerate(zip(Bs, ranks)):
            want = (r, n * (n + 1) // 2) if packed else (r, n, n)
            if tuple(B.shape) != want or B.dtype != torch.complex128:
                raise ValueError("instance %d: B[%d] must be complex128 %s%s"
                                 % (i, t, list(want), " (packed layout)" if packed else ""))
        if c is not None and (c.dtype != torch.complex128 or c.dim() not in (1, 2)
                              or c.shape[-1] != info.n_ref or c.numel() == 0):
            raise ValueError("instance %d: c must be complex128 [N_P = %d] (or [n_roots, N_P])" % (i, info.n_ref))

    def energy(self, insts, parts=True):
        """insts: list of (h, [B_t], c) complex128 device tensors per
        instance.  Returns the device tensor of E2 per instance (and the
        per-class parts when parts=True)."""
        arr, keep = self._inputs(insts)
        code = capi.lib().mrpt2_energy(self.plan.handle, arr, self.persistent.data_ptr(),
                                       self.workspace.data_ptr(), self.plan.workspace_bytes, self._sptr(),
                                       self.e2.data_ptr(), self.parts.data_ptr() if parts else None)
        capi.check(code, "mrpt2_energy")
        del keep
        return (self.e2, self.parts) if parts else self.e2

    def energy_roots(self, insts):
        """State-specific E2 of several reference states at once: insts is a
        list of (h, [B_t], C) per instance with C complex128 of shape
        [n_roots, N_P] (the same n_roots for every instance).  The integral
        build runs once; returns E2 [n_roots, n_inst] and the per-class
        parts [n_roots, n_inst, 12] (device tensors)."""
        torch = self.torch
        shapes = {tuple(c.shape) for _, _, c in insts}
        if any(len(sh) != 2 for sh in shapes) or len({sh[0] for sh in shapes}) != 1:
            raise ValueError("every C must be [n_roots, N_P] with one n_roots")
        n_roots = next(iter(shapes))[0]
        arr, keep = self._inputs(insts)
        e2 = torch.zeros((n_roots, self.plan.n_inst), dtype=torch.float64, device=self.device)
        parts = torch.zeros((n_roots, self.plan.n_inst, 12), dtype=torch.float64, device=self.device)
        code = capi.lib().mrpt2_energy_roots(self.plan.handle, arr, n_roots, self.persistent.data_ptr(),
                                             self.workspace.data_ptr(), self.plan.workspace_bytes, self._sptr(),
                                             e2.data_ptr(), parts.data_ptr())
        capi.check(code, "mrpt2_energy_roots")
        del keep
        return e2, parts

    def energy_async(self, insts, stream=None):
        """Enqueue an evaluation without synchronising (capturable in a HIP
        graph).  The input tensors must stay alive until it has run; call
        check() to read the error flag."""
        arr, keep = self._inputs(insts)
        s = ctypes.c_void_p((stream or self.stream).cuda_stream)
        code = capi.lib().mrpt2_energy_async(self.plan.handle, arr, self.persistent.data_ptr(),
                                             self.workspace.data_ptr(), self.plan.workspace_bytes, s,
                                             self.e2.data_ptr(), self.parts.data_ptr())
        capi.check(code, "mrpt2_energy_async")
        self._keep = keep
        return self.e2, self.parts

    def check(self, stream=None):
        s = ctypes.c_void_p((stream or self.stream).cuda_stream)
        capi.check(capi.lib().mrpt2_check(self.plan.handle, self.workspace.data_ptr(), s), "mrpt2_check")

    def energy_timed(self, insts):
        """energy() with per-stage milliseconds (dict over capi.STAGES)."""
        arr, keep = self._inputs(insts)
        ms = (ctypes.c_float * capi.N_STAGE)()
        code = capi.lib().mrpt2_energy_timed(self.plan.handle, arr, self.persistent.data_ptr(),
                                             self.workspace.data_ptr(), self.plan.workspace_bytes, self._sptr(),
                                             self.e2.data_ptr(), self.parts.data_ptr(), ms)
        capi.check(code, "mrpt2_energy_timed")
        del keep
        return self.e2, self.parts, dict(zip(capi.STAGES, list(ms)))

    def backward(self, insts, grad_e2=None, timed=False, asynchronous=False, stream=None):
        """Gradients of E2 for every instance: list of (dh, [dB_t], dc)
        complex128 device tensors (dh, dB Hermitian-projected), and the
        device tensor of E2 per instance.  grad_e2: device float64 [n_inst]
        upstream gradients (ones when None).  The gradient workspace is
        allocated on first use and kept.  asynchronous=True enqueues the
        whole call on `stream` without synchronising (capturable in a HIP
        graph with the forward recomputation; read the flag with check());
        the inputs, grad_e2 and the returned tensors must then stay alive
        until it has run."""
        torch = self.torch
        if getattr(self, "grad_workspace", None) is None:
            self.grad_workspace = torch.empty(max(self.plan.grad_bytes, 256), dtype=torch.uint8,
                                              device=self.device)
        if grad_e2 is None:
            grad_e2 = torch.ones(self.plan.n_inst, dtype=torch.float64, device=self.device)
        grad_e2 = grad_e2.to(device=self.device, dtype=torch.float64).contiguous()
        if grad_e2.numel() != self.plan.n_inst:
            raise ValueError("grad_e2 must hold one value per instance (%d), got %d"
                             % (self.plan.n_inst, grad_e2.numel()))
        arr, keep = self._inputs(insts)
        outs = []
        garr = (capi.Grads * len(insts))()
        for i, (h, Bs, c) in enumerate(insts):
            dh = torch.empty_like(h)
            dBs = [torch.empty_like(B) for B in Bs]
            dc = torch.empty_like(c)
            garr[i].dh = dh.data_ptr()
            for t, dB in enumerate(dBs):
                garr[i].dB[t] = dB.data_ptr()
            garr[i].dc = dc.data_ptr()
            outs.append((dh, dBs, dc))
        sptr = ctypes.c_void_p((stream or self.stream).cuda_stream) if asynchronous else self._sptr()
        args = (self.plan.handle, arr, self.persistent.data_ptr(), self.workspace.data_ptr(),
                self.plan.workspace_bytes, self.grad_workspace.data_ptr(), self.plan.grad_bytes,
                grad_e2.data_ptr(), garr, sptr, self.e2.data_ptr())
        if asynchronous:
            capi.check(capi.lib().mrpt2_energy_backward_async(*args), "mrpt2_energy_backward_async")
            self._keep = (keep, grad_e2)
            return outs, self.e2
        if timed:
            ms = (ctypes.c_float * capi.N_STAGE_B)()
            capi.check(capi.lib().mrpt2_energy_backward_timed(*args, ms), "mrpt2_energy_backward_timed")
            del keep
            return outs, self.e2, dict(zip(capi.STAGES_B, list(ms)))
        capi.check(capi.lib().mrpt2_energy_backward(*args), "mrpt2_energy_backward")
        del keep
        return outs, self.e2

    def delta_stats(self, insts, thresh=0.0):
        """Smallest |E0 - H_KK| per instance and excitation class and the
        number of external determinants with |E0 - H_KK| < thresh (host numpy
        [n_inst, 9] float64 and int64; class order of capi.Info)."""
        arr, keep = self._inputs(insts)
        n = self.plan.n_inst
        mn = np.zeros((n, capi.N_CLASS))
        cnt = np.zeros((n, capi.N_CLASS), dtype=np.int64)
        code = capi.lib().mrpt2_delta_stats(self.plan.handle, arr, self.persistent.data_ptr(),
                                            self.workspace.data_ptr(), self.plan.workspace_bytes, self._sptr(),
                                            float(thresh), mn.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                            cnt.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)))
        capi.check(code, "mrpt2_delta_stats")
        del keep
        return mn, cnt

    def class_partials(self, cls, inst=0):
        """Block partial sums of class cls from the last energy() (host numpy,
        not divided by ||C||^2)."""
        n = self.plan.class_blocks(cls, inst)
        out = np.zeros(max(n, 1))
        capi.check(capi.lib().mrpt2_class_partials(self.plan.handle, inst, cls, self.workspace.data_ptr(),
                                                   self._sptr(),
                                                   out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))),
                   "mrpt2_class_partials")
        return out[:n]

    def reference_states(self, h, Bs, k=1, tol=1e-10, max_iter=500, inst=0, direct=False):
        """The k lowest eigenpairs of H_PP - E_core by the library's block
        Davidson solver on the device: C [k, N_P] complex128 device tensor in
        plan order (unit norm, largest component real positive), energies
        (host numpy, ascending) and the iteration count.  direct=True applies
        H_PP by the direct sigma-build in P (excitation lists, no stored
        H_PP) instead of a dense H_PP."""
        torch = self.torch
        n_p = self.plan.info(inst).n_ref
        nbytes = ctypes.c_size_t()
        size_fn = "mrpt2_reference_states_direct_size" if direct else "mrpt2_reference_states_size"
        capi.check(getattr(capi.lib(), size_fn)(self.plan.handle, inst, k, ctypes.byref(nbytes)), size_fn)
        dv = torch.empty(max(nbytes.value, 256), dtype=torch.uint8, device=self.device)
        C = torch.empty((k, n_p), dtype=torch.complex128, device=self.device)
        e = np.zeros(k)
        its = ctypes.c_int32()
        arr, keep = self._inputs([(h, Bs, None)], inst=inst)
        fn = "mrpt2_reference_states_direct" if direct else "mrpt2_reference_states"
        code = getattr(capi.lib(), fn)(self.plan.handle, inst, arr, k, tol, max_iter,
                                       self.persistent.data_ptr(), self.workspace.data_ptr(),
                                       self.plan.workspace_bytes, dv.data_ptr(), nbytes.value,
                                       self._sptr(), C.data_ptr(), e.ctypes.data, ctypes.byref(its))
        capi.check(code, fn)
        del keep, dv
        return C, e, its.value

    def reference_sigma(self, h, Bs, X, inst=0):
        """(H_PP - E_core) X for the rows of X (complex128 [m, N_P] device
        tensor, plan order) by the direct sigma-build in P: excitation lists
        of the reference space, elements from the Slater-Condon rules, no
        stored H_PP."""
        torch = self.torch
        n_p = self.plan.info(inst).n_ref
        X = X.reshape(-1, n_p) if X.dim() == 1 else X
        if X.dtype != torch.complex128 or X.shape[-1] != n_p or not X.is_contiguous() or X.device != self.device:
            raise ValueError("X must be a contiguous complex128 [m, %d] tensor on the engine's device" % n_p)
        Y = torch.empty_like(X)
        arr, keep = self._inputs([(h, Bs, None)], inst=inst)
        code = capi.lib().mrpt2_reference_sigma(self.plan.handle, inst, arr, X.shape[0], X.data_ptr(),
                                                self.persistent.data_ptr(), self.workspace.data_ptr(),
                                                self.plan.workspace_bytes, self._sptr(), Y.data_ptr())
        capi.check(code, "mrpt2_reference_sigma")
        del keep
        return Y

    def reference_hamiltonian(self, h, Bs, inst=0):
        torch = self.torch
        n_p = self.plan.info(inst).n_ref
        out = torch.empty((n_p, n_p), dtype=torch.complex128, device=self.device)
        arr, keep = self._inputs([(h, Bs, None)], inst=inst)
        code = capi.lib().mrpt2_reference_hamiltonian(self.plan.handle, inst, arr, self.persistent.data_ptr(),
                                                      self.workspace.data_ptr(), self.plan.workspace_bytes,
                                                      self._sptr(), out.data_ptr())
        capi.check(code, "mrpt2_reference_hamiltonian")
        del keep
        return out


def hermitian_eigh(a):
    """Eigenpairs (ascending) of a small complex Hermitian host matrix with the
    library's Jacobi solver (the one its Davidson solver uses)."""
    a = np.ascontiguousarray(a, dtype=np.complex128)
    n = a.shape[0]
    w = np.zeros(n)
    v = np.zeros((n, n), dtype=np.complex128)
    capi.check(capi.lib().mrpt2_hermitian_eigh(n, a.ctypes.data, w.ctypes.data, v.ctypes.data),
               "mrpt2_hermitian_eigh")
    return w, v


def _autograd_function():
    import torch

    class EnergyFn(torch.autograd.Function):
        """E2 of one instance as a differentiable function of (h, B_1..B_k, c).
        The forward pass runs mrpt2_energy; the backward pass runs
        mrpt2_energy_backward (which recomputes the forward pass and the
        first-order vector block by block).  Gradients follow torch's
        convention for complex inputs; dh and dB are Hermitian-projected."""

        @staticmethod
        def forward(ctx, engine, h, c, *Bs):
            e2 = engine.energy([(h, list(Bs), c)], parts=False)[0].clone()
            ctx.engine = engine
            ctx.save_for_backward(h, c, *Bs)
            return e2

        @staticmethod
        def backward(ctx, grad):
            h, c, *Bs = ctx.saved_tensors
            g = grad.reshape(1).to(torch.float64).contiguous()
            (dh, dBs, dc), = ctx.engine.backward([(h, list(Bs), c)], g)[0]
            return (None, dh, dc, *dBs)

    return EnergyFn


_ENERGY_FN = None


def energy(engine, h, Bs, c):
    """Differentiable E2 (torch autograd) of a one-instance engine."""
    global _ENERGY_FN
    if _ENERGY_FN is None:
        _ENERGY_FN = _autograd_function()
    return _ENERGY_FN.apply(engine, h, c, *Bs)
