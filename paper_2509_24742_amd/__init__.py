"""SRBE constant-potential step on AMD MI355X (gfx950).

The compute path is libsrbe.so (hand-written HIP kernels behind the C ABI in
include/srbe.h).  ``binding`` exposes that ABI function by function; ``System``
below is a convenience wrapper that allocates the outputs with torch.  Importing
this package does not load the library; the first call does, and raises if the
library has not been built.
"""

import numpy as np

from . import binding
from .binding import (SRBE_BF16, SRBE_FLAG_ENERGY_PARTS, SRBE_FLAG_IID_SAMPLER, SRBE_FLAG_KSPACE_ONLY, SRBE_FLAG_LATTICE_SOLVE, SRBE_FLAG_NO_CP, SRBE_FP32, SRBE_FP64, SrbeError, srbe_create, srbe_destroy,  # noqa: F401
                      srbe_error_string, srbe_graph_create, srbe_graph_destroy, srbe_graph_launch,
                      srbe_graph_set_step, srbe_last_error, srbe_n_ele, srbe_normaliser, srbe_phase_name,
                      srbe_profile_enable, srbe_profile_read, srbe_sample, srbe_step, srbe_sync_status,
                      SRBE_TUNE_NAMES, srbe_electrode_forces, srbe_get_tuning, srbe_langevin_update, srbe_set_tuning,
                      srbe_tune)


class System:
    """One electrode geometry (a handle) plus output allocation for steps over replicas."""

    def __init__(self, params, ele_pos, ele_side, flags=0):
        self.params = dict(params)
        self.flags = int(flags)
        self.h = srbe_create(self.params, ele_pos, ele_side, flags=flags)
        self.n_ele = srbe_n_ele(self.h)
        self.G = srbe_normaliser(self.h)

    def close(self):
        if self.h is not None:
            srbe_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def outputs(self, ion_offsets, device, want_b=True, want_kset=True):
        """Output tensors of a step over the given replicas (Q, F, b, psibar, E, kset)."""
        import torch
        off = np.asarray(ion_offsets, dtype=np.int64)
        R = len(off) - 1
        N = int(off[-1])
        P = int(self.params["P"])
        return dict(
            Q=torch.empty(R * self.n_ele, dtype=torch.float64, device=device),
            F=torch.empty(3 * N, dtype=torch.float64, device=device),
            b=torch.empty(R * self.n_ele, dtype=torch.float64, device=device) if want_b else None,
            psibar=torch.empty(R, dtype=torch.float64, device=device),
            # with SRBE_FLAG_ENERGY_PARTS: [total, real, fourier, self, slab] per replica
            E=torch.empty(R * (5 if self.flags & SRBE_FLAG_ENERGY_PARTS else 1), dtype=torch.float64,
                          device=device),
            kset=torch.empty(R * P * 3, dtype=torch.int32, device=device) if (want_kset and P) else None,
        )

    def tune(self, ion_offsets, ion_xyz, ion_q, dpsi, seed, precision=SRBE_FP64, iters=10, cache=None,
             tune_missing=True):
        """Choose the launch parameters for this batch shape (srbe_tune) and keep them in the handle.

        cache: path of a JSON file of earlier choices, keyed by device architecture, precision,
        replica count, largest replica, electrode count and P; a hit is applied without timing
        and a miss is timed and added (with tune_missing false, a miss keeps the defaults and
        nothing is timed or written).  Returns dict(params, ms_default, ms_tuned, cached).
        srbe_tune's live timing is switched off at present, so a miss with tune_missing true
        raises SrbeError.
        """
        import json
        import os
        import torch
        off = np.asarray(ion_offsets, dtype=np.int64)
        key = None
        entries = {}
        if cache is not None:
            arch = torch.cuda.get_device_properties(dpsi.device).gcnArchName
            key = (f"{arch}|{'fp32' if precision == SRBE_FP32 else 'fp64'}|R={len(off) - 1}|"
                   f"maxrep={int(np.diff(off).max()) if len(off) > 1 else 0}|n_ele={self.n_ele}|P={self.params['P']}")
            if os.path.exists(cache):
                with open(cache) as f:
                    entries = json.load(f)
            if key in entries:
                # a parameter the entry predates keeps the value the library would choose
                dflt = dict(zip(SRBE_TUNE_NAMES, srbe_get_tuning(self.h, precision, off)))
                params = [int(entries[key]["params"].get(name, dflt[name])) for name in SRBE_TUNE_NAMES]
                srbe_set_tuning(self.h, precision, off, params)
                return dict(params=params, ms_default=entries[key].get("ms_default"),
                            ms_tuned=entries[key].get("ms_tuned"), cached=True)
        if not tune_missing:
            return dict(params=srbe_get_tuning(self.h, precision, off), ms_default=None, ms_tuned=None,
                        cached=False)
        params, ms0, ms1 = srbe_tune(self.h, precision, off, ion_xyz, ion_q, dpsi, seed, iters=iters)
        if cache is not None:
            entries[key] = dict(params=dict(zip(SRBE_TUNE_NAMES, params)), ms_default=ms0, ms_tuned=ms1)
            tmp = cache + ".tmp"
            with open(tmp, "w") as f:
                json.dump(entries, f, indent=1, sort_keys=True)
            os.replace(tmp, cache)
        return dict(params=params, ms_default=ms0, ms_tuned=ms1, cached=False)

    def capture(self, ion_offsets, ion_xyz, ion_q, dpsi, seed, first_step, precision=SRBE_FP64, kset_in=None,
                Q_in=None, want_b=True, want_kset=True, out=None):
        """Capture one step with fixed buffers; returns a StepGraph (replay with .launch())."""
        off = np.asarray(ion_offsets, dtype=np.int64)
        if out is None:
            out = self.outputs(off, dpsi.device, want_b, want_kset)
        gr = srbe_graph_create(self.h, precision, off, ion_xyz, ion_q, dpsi, seed, first_step, out["Q"], out["F"],
                               kset_in=kset_in, Q_in=Q_in, b_out=out["b"], psibar_out=out["psibar"],
                               energy_out=out["E"], kset_out=out["kset"])
        # the graph keeps raw pointers: hold the inputs and outputs for its lifetime
        return StepGraph(self, gr, out, (ion_xyz, ion_q, dpsi, seed, kset_in, Q_in))

    def step(self, ion_offsets, ion_xyz, ion_q, dpsi, seed, step, precision=SRBE_FP64, kset_in=None, Q_in=None,
             want_b=True, want_kset=True, out=None, stream=None):
        """Run one step; returns a dict of CUDA tensors (Q, F, b, psibar, E, kset)."""
        off = np.asarray(ion_offsets, dtype=np.int64)
        if out is None:
            out = self.outputs(off, dpsi.device, want_b, want_kset)
        srbe_step(self.h, precision, off, ion_xyz, ion_q, dpsi, seed, step, out["Q"], out["F"], kset_in=kset_in,
                  Q_in=Q_in, b_out=out["b"], psibar_out=out["psibar"], energy_out=out["E"], kset_out=out["kset"],
                  stream=stream)
        return out


class StepGraph:
    """A captured step: launch() replays it (the step counter advances by one per replay)."""

    def __init__(self, system, gr, out, inputs):
        self.system = system
        self.gr = gr
        self.out = out
        self._inputs = inputs

    def launch(self, stream=None):
        srbe_graph_launch(self.gr, stream)
        return self.out

    def set_step(self, step, stream=None):
        srbe_graph_set_step(self.gr, step, stream)

    def close(self):
        if self.gr is not None:
            srbe_graph_destroy(self.gr)
            self.gr = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
