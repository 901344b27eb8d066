"""Sim: a batch of gel/indenter environments stepped on the GPU through libt2r.

Torch provides the device buffers and the stream; all compute is in the HIP
library. Typical use:

    sim = Sim.from_workload(workload, opts)
    for s in range(1, S + 1):
        markers, status = sim.step(poses[:, s])   # poses as a (n_env, 7) tensor
"""

from __future__ import annotations

import atexit
import os
import weakref

import numpy as np
import torch

from . import t2r


_LIVE = weakref.WeakSet()
# autotune results of this process, keyed by Sim.tune_key
_TUNE_CACHE: dict = {}


@atexit.register
def _close_all():
    # contexts still open at exit give their memory back to torch's allocator
    # while torch is still there
    for sim in list(_LIVE):
        sim.close()


class Sim:
    def __init__(self, opts: t2r.SolverOpts | None = None, device: str | int = "cuda:0", stream=None,
                 torch_memory: bool = True):
        """stream: the torch stream the library enqueues on (default: the current
        stream; graph_step needs a non-default one, e.g. torch.cuda.Stream()).
        torch_memory: every device allocation of the library comes from torch's
        caching allocator on that stream (t2r_set_allocator), so torch owns all
        device memory; False lets the library call hipMalloc itself."""
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.ctx = t2r.Context(opts, self.stream.cuda_stream)
        if torch_memory:
            dev = self.device.index if self.device.index is not None else torch.cuda.current_device()
            stream_handle = self.stream.cuda_stream

            def alloc(nbytes):
                try:
                    return torch.cuda.caching_allocator_alloc(nbytes, dev, stream_handle)
                except RuntimeError:
                    return 0  # out of memory: the library reports T2R_E_NOMEM

            self.ctx.set_allocator(alloc, torch.cuda.caching_allocator_delete)
        _LIVE.add(self)
        self._graph = None
        self._graph_gen = -1
        self.mats = []
        self.gel_ids = {}
        self.ind_ids = {}
        self.env_gel = []
        self.env_ind = []
        self.ind_sizes = {}
        self.n_m = []
        self.n_v = []

    @classmethod
    def from_workload(cls, workload, opts: t2r.SolverOpts | None = None, device="cuda:0",
                      envs=None, stream=None, torch_memory: bool = True):
        """Builds every gel and indenter class of a scenes.Workload and its envs
        (all of them, or the listed indices)."""
        sim = cls(opts, device, stream, torch_memory=torch_memory)
        for name, g in workload.meshes.items():
            sim.gel_ids[name] = sim.ctx.add_gel(g.X, g.tets, g.fixed, g.markers)
        for name, ind in workload.indenters.items():
            sim.ind_ids[name] = sim.ctx.add_indenter(ind.Y, ind.tris)
            sim.ind_sizes[sim.ind_ids[name]] = (int(len(ind.Y)), int(len(ind.tris)))
        sel = workload.envs if envs is None else [workload.envs[i] for i in envs]
        sim.ctx.add_envs([sim.gel_ids[e.mesh] for e in sel], [sim.ind_ids[e.indenter] for e in sel],
                         [e.material() for e in sel], np.stack([e.poses[0] for e in sel]))
        sim.env_gel = [sim.gel_ids[e.mesh] for e in sel]
        sim.env_ind = [sim.ind_ids[e.indenter] for e in sel]
        sim.mats = [e.material() for e in sel]
        for e in sel:
            info = sim.ctx.gel_info(sim.gel_ids[e.mesh])
            sim.n_m.append(info["n_m"])
            sim.n_v.append(info["n_v"])
        sim.n_env = len(sel)
        sim.markers = torch.zeros((sum(sim.n_m), 3), dtype=torch.float64, device=sim.device)
        sim.x = torch.zeros((sum(sim.n_v), 3), dtype=torch.float64, device=sim.device)
        sim.status = torch.zeros(sim.n_env, dtype=torch.int32, device=sim.device)
        return sim

    def step(self, poses, mask=None, want_x=False):
        """One load step of every env to `poses` ((n_env, 7), any float array).
        Returns (markers tensor (sum n_m, 3), status tensor (n_env,)), not synchronised."""
        p = torch.as_tensor(np.asarray(poses, dtype=np.float64) if not torch.is_tensor(poses) else poses,
                            dtype=torch.float64, device=self.device).contiguous()
        m = None if mask is None else torch.as_tensor(mask, dtype=torch.int32, device=self.device)
        self.ctx.step(p, m, self.markers, self.x if want_x else None, self.status)
        return self.markers, self.status

    def step_sequence(self, poses, mask=None, want_x=False):
        """Load steps k = 0..S-1 of every env to poses[k] ((S, n_env, 7)) in one launch.
        Returns (markers tensor (S, sum n_m, 3), status tensor (S, n_env)), not synchronised."""
        p = torch.as_tensor(np.asarray(poses, dtype=np.float64) if not torch.is_tensor(poses) else poses,
                            dtype=torch.float64, device=self.device).contiguous()
        n_steps = p.shape[0]
        m = None if mask is None else torch.as_tensor(mask, dtype=torch.int32, device=self.device)
        markers = torch.zeros((n_steps, sum(self.n_m), 3), dtype=torch.float64, device=self.device)
        status = torch.zeros((n_steps, self.n_env), dtype=torch.int32, device=self.device)
        self.ctx.step_sequence(n_steps, p, m, markers, self.x if want_x else None, status)
        return markers, status

    def backward(self, dL_du):
        """dL/dtheta (n_env, 9) of a loss on the current markers: theta = (E, nu, mu_f,
        dt (3), dw (3)) per env (see t2r_backward). dL_du: (sum n_m, 3). Not synchronised."""
        g = torch.as_tensor(dL_du, dtype=torch.float64, device=self.device).contiguous()
        out = torch.zeros((self.n_env, 9), dtype=torch.float64, device=self.device)
        self.ctx.backward(g, out)
        return out

    def save_checkpoint(self):
        """A device copy of everything later load steps read besides their inputs
        (see t2r_save_checkpoint). Not synchronised."""
        buf = torch.empty(self.ctx.checkpoint_size(), dtype=torch.float64, device=self.device)
        self.ctx.save_checkpoint(buf)
        return buf

    def load_checkpoint(self, buf):
        """Restores a save_checkpoint copy (same meshes and envs)."""
        self.ctx.load_checkpoint(torch.as_tensor(buf, device=self.device).contiguous())

    def record(self, max_steps):
        """Starts a trajectory tape of at most max_steps load steps from the current
        state (0 stops recording); see t2r_record."""
        self.ctx.record(max_steps)

    def tape_state(self, entry):
        """Positions (sum n_v, 3) and poses (n_env, 7) of tape entry `entry` (see
        t2r_tape_read), as host arrays (synchronises this Sim's stream)."""
        import numpy as np
        st = torch.empty(self.ctx.state_size(), dtype=torch.float64, device=self.device)
        self.ctx.tape_read(entry, st)
        self.stream.synchronize()
        a = st.cpu().numpy()
        xs, qs, off = [], [], 0
        for nv in self.n_v:
            xs.append(a[off:off + 3 * nv].reshape(nv, 3))
            qs.append(a[off + 3 * nv:off + 3 * nv + 7])
            off += 3 * nv + 7
        return np.concatenate(xs), np.stack(qs)

    def backward_sequence(self, dL_du):
        """dL/dtheta (n_env, 9) of a loss on the markers of the last S recorded load
        steps; dL_du: (S, sum n_m, 3), oldest step first (see t2r_backward_sequence).
        Not synchronised."""
        g = torch.as_tensor(dL_du, dtype=torch.float64, device=self.device).contiguous()
        out = torch.zeros((self.n_env, 9), dtype=torch.float64, device=self.device)
        self.ctx.backward_sequence(g.shape[0], g, out)
        return out

    def graph_step(self, poses):
        """One load step of every env, replayed from a captured HIP graph.

        The first call runs the step eagerly (so that every device buffer exists)
        and then captures the library's launches for one step (env ordering and
        the step kernel) on this Sim's stream; later calls copy `poses` into the
        captured pose buffer and replay. Needs a non-default stream. Returns
        (markers, status) like step(), not synchronised."""
        if self.ctx.tape_length() >= 0:
            raise RuntimeError("graph_step cannot record a tape (a replay would rewrite one entry); "
                               "stop recording with record(0) or use step()")
        p = torch.as_tensor(np.asarray(poses, dtype=np.float64) if not torch.is_tensor(poses) else poses,
                            dtype=torch.float64, device=self.device)
        if self._graph is not None and self._graph_gen != self.ctx.layout_generation():
            self._graph = None  # buffers or options changed since the capture: capture again
        with torch.cuda.stream(self.stream):
            if self._graph is None:
                self._pose_buf = p.clone().contiguous()
                self.ctx.step(self._pose_buf, None, self.markers, None, self.status)
                self.stream.synchronize()
                graph = torch.cuda.CUDAGraph()
                with torch.cuda.graph(graph, stream=self.stream):
                    self.ctx.step(self._pose_buf, None, self.markers, None, self.status)
                self._graph = graph
                self._graph_gen = self.ctx.layout_generation()
            else:
                self._pose_buf.copy_(p)
                self._graph.replay()
        return self.markers, self.status

    def tune_key(self, target_steps=1) -> str:
        """Cache key of an autotune result: the device, the launch length and the
        batch's composition (count of envs per gel class and indenter class, each
        class by its sizes)."""
        import collections
        comp = collections.Counter()
        for g, i in zip(self.env_gel, self.env_ind):
            info = self.ctx.gel_info(g)
            comp[(info["n_v"], info["n_t"], info["n_sf"]) + tuple(self.ind_sizes.get(i, (0, 0)))] += 1
        name = torch.cuda.get_device_name(self.device)
        return repr((name, int(target_steps), sorted(comp.items())))

    def autotune(self, poses, blocks=(256, 512), target_steps=1, cache=True, cache_path=None):
        """Picks the workgroup shape and pair-list capacity for this batch.

        With cache, a batch of the same composition on the same device and launch
        length reuses an earlier result without trial launches: from this process
        (a module-level table) or from the JSON file cache_path (read if it
        exists, written after a tuning run).

        Runs the trial load steps `poses` ((S, n_env, 7)) from the current state
        once per candidate block shape and keeps the faster one for launches of
        `target_steps` load steps: short launches are judged by their measured
        duration; long ones (>= 4 steps) by the larger of the slowest env and
        the summed env time over the resident workgroup slots (2 per CU at 256
        threads, 1 at 512), since their imbalance averages out. Doubles the
        pair capacity while any list of the trial used more than half of it,
        and restores the state (positions and poses). Tuning time is setup, not
        part of a timed step. Returns {"block_size", "pair_capacity",
        "trial_ms", "predicted_ms", "list_fill"}."""
        import json
        import time
        key = self.tune_key(target_steps) if cache else None
        if cache and cache_path and key not in _TUNE_CACHE and os.path.exists(cache_path):
            with open(cache_path) as fh:
                _TUNE_CACHE.update(json.load(fh))
        if cache and key in _TUNE_CACHE:
            hit = _TUNE_CACHE[key]
            opts = self.ctx.get_opts()
            opts.block_size = hit["block_size"]
            opts.pair_capacity = hit["pair_capacity"]
            self.ctx.set_opts(opts)
            return dict(hit, cached=True)
        saved = torch.empty(self.ctx.state_size(), dtype=torch.float64, device=self.device)
        self.ctx.get_state(saved)
        opts = self.ctx.get_opts()
        n_cu = torch.cuda.get_device_properties(self.device).multi_processor_count
        trial_ms, predicted, used = {}, {}, 0.0
        for b in blocks:
            opts.block_size = b
            self.ctx.set_opts(opts)
            self.ctx.set_state(saved)
            self.stream.synchronize()
            t0 = time.perf_counter()
            self.step_sequence(poses)
            self.stream.synchronize()
            trial_ms[b] = 1e3 * (time.perf_counter() - t0)
            st = self.stats()
            env_ms = [x["phase_ms"][8] for x in st]
            slots = n_cu * (2 if b == 256 else 1)
            predicted[b] = (max(max(env_ms), sum(env_ms) / slots) if target_steps >= 4 else trial_ms[b])
            used = max([used] + [x["list_fill"] for x in st])
        opts.block_size = min(predicted, key=predicted.get)
        grow = 1
        while used > 0.5:
            grow, used = 2 * grow, used / 2
        if grow > 1:
            # automatic capacities differ per gel class; a fixed one takes the largest, grown
            base = max(self.ctx.gel_info(g)["pair_capacity"] for g in set(self.env_gel))
            opts.pair_capacity = grow * base
        self.ctx.set_opts(opts)
        self.ctx.set_state(saved)
        self.stream.synchronize()
        out = {"block_size": opts.block_size, "pair_capacity": opts.pair_capacity, "trial_ms": trial_ms,
               "predicted_ms": predicted, "list_fill": used * grow}
        if cache:
            _TUNE_CACHE[key] = out
            if cache_path:
                with open(cache_path, "w") as fh:
                    json.dump(_TUNE_CACHE, fh, indent=1)
        return dict(out, cached=False)

    def close(self):
        """Releases the library's device memory (back to torch's allocator)."""
        self._graph = None
        self.ctx.close()

    def split_markers(self, markers=None):
        markers = self.markers if markers is None else markers
        return torch.split(markers, self.n_m)

    def split_x(self, x=None):
        x = self.x if x is None else x
        return torch.split(x, self.n_v)

    def stats(self):
        return self.ctx.get_stats()
