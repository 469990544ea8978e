"""Continuous batching of P_ell requests of one shape (many mocks of one
survey, the covariance use of Sec. III.C).

A ``BatchServer`` owns ``groups`` groups of ``group_size`` plans (one
configuration, a workspace each, one HIP stream per group).  ``submit``
queues a request; ``poll`` completes the batches whose events have fired
(copying their results out of the plans' page-locked output arrays) and
hands every free group the queued requests, up to ``group_size`` of them, as
one ``frsd_pk_batch``.  Requests that arrive while a batch runs therefore
form the next batch, and the groups overlap on the device.  With
``group_size = 1`` the same loop serves one request per launch on each
stream.

With a random catalogue (``randoms``), every plan holds its spectra
(``frsd_random_cache``) and requests carry galaxies and alpha only;
otherwise each request carries its own randoms.  Catalogues are device (or
page-locked host) tensors as ``fastrsd.device_catalog`` makes them; they must
stay unchanged until their request completes.
"""

from __future__ import annotations

import time
from collections import deque
from dataclasses import dataclass, field

import torch

from . import fastrsd as F


@dataclass
class Request:
    rid: int
    gal: dict
    alpha: float
    ran: dict | None = None
    t_submit: float = 0.0
    t_done: float = 0.0
    result: dict = field(default_factory=dict)


class BatchServer:
    def __init__(self, cfg: F.Config, groups: int = 2, group_size: int = 8, device="cuda",
                 randoms: dict | None = None):
        if not 1 <= group_size <= F.FRSD_MAX_BATCH:
            raise ValueError(f"group_size must be 1..{F.FRSD_MAX_BATCH}")
        if randoms is not None and not cfg.random_cache:
            raise ValueError("a shared random catalogue needs a configuration with random_cache")
        self.device = torch.device(device)
        self.cached = randoms is not None
        self.groups = []
        for _ in range(groups):
            stream = torch.cuda.Stream(self.device)
            plans = [F.Plan(cfg, device=self.device, stream=stream, host_outputs=True) for _ in range(group_size)]
            if randoms is not None:
                for pl in plans:
                    pl.random_cache(randoms)
            self.groups.append({"plans": plans, "stream": stream, "event": None, "reqs": []})
        self._randoms = randoms
        self.queue: deque[Request] = deque()
        self.next_id = 0
        self.batch_sizes: list[int] = []

    @property
    def workspace_bytes(self) -> int:
        return sum(pl.ws_bytes for g in self.groups for pl in g["plans"])

    def submit(self, gal: dict, alpha: float, ran: dict | None = None) -> Request:
        if self.cached == (ran is not None):
            raise ValueError("requests carry randoms exactly when the server holds no random catalogue")
        req = Request(self.next_id, gal, float(alpha), ran, time.perf_counter())
        self.next_id += 1
        self.queue.append(req)
        return req

    def _launch(self, g: dict) -> None:
        n = min(len(self.queue), len(g["plans"]))
        reqs = [self.queue.popleft() for _ in range(n)]
        plans = g["plans"][:n]
        F.pk_batch(plans, [r.gal for r in reqs], None if self.cached else [r.ran for r in reqs],
                   [r.alpha for r in reqs])
        ev = torch.cuda.Event()
        ev.record(g["stream"])
        g["event"], g["reqs"] = ev, reqs
        self.batch_sizes.append(n)

    def poll(self) -> list[Request]:
        """Complete finished batches and launch queued requests on free groups;
        returns the requests completed by this call."""
        done = []
        for g in self.groups:
            if g["event"] is not None and g["event"].query():
                t = time.perf_counter()
                for pl, req in zip(g["plans"], g["reqs"]):
                    req.result = {k: v.numpy().copy() for k, v in pl.pk_buf.items()}
                    req.t_done = t
                done.extend(g["reqs"])
                g["event"], g["reqs"] = None, []
            if g["event"] is None and self.queue:
                self._launch(g)
        return done

    def busy(self) -> bool:
        return bool(self.queue) or any(g["event"] is not None for g in self.groups)

    def drain(self) -> list[Request]:
        """poll until every submitted request has completed."""
        done = []
        while self.busy():
            done.extend(self.poll())
        return done

    def rejected(self) -> int:
        """Objects rejected by the last batch of every plan (frsd_status; synchronises)."""
        return sum(pl.status() for g in self.groups for pl in g["plans"])
