"""TNS of a timed design as a differentiable function (torch.autograd.Function).

Forward: the library's propagation and slack passes on the given net delays and driver
loads (device tensors in the graph's internal order) give TNS per view.  Backward: the
library's argmax-routed adjoint (sta_tns_adjoint) gives dTNS/d(net delay) per sink arc and
dTNS/d(load) per driver; autograd's incoming weights per view are applied to them."""
from __future__ import annotations

import torch

from . import sta


class TimedDesign:
    """An uploaded graph with its library, views, primary-input and endpoint data, and the
    device buffers the forward pass fills."""

    def __init__(self, g: sta.Graph, lib: sta.LibraryC, views: sta.ViewsC, pi_ts, ep_rat, net_imp2):
        self.g, self.lib, self.views = g, lib, views
        self.pi_ts, self.ep_rat = pi_ts, ep_rat
        self.nd = sta.alloc_net(g)
        self.nd["net_imp2"].copy_(net_imp2)
        self.tm = sta.alloc_timing(g, views.n_views)
        self.sl = sta.alloc_slack(g, views.n_views)
        self.adj = sta.alloc_adjoint(g, views.n_views)
        self.run = 0          # forward passes made on these buffers

    def evaluate(self, net_delay, load) -> int:
        """Fills the buffers for (net_delay, load): propagation and slack; returns the
        pass number the buffers now hold."""
        self.nd["net_delay"].copy_(net_delay)
        self.nd["load"].copy_(load)
        sta.arc_load(self.g, self.nd)
        sta.propagate(self.g, self.lib, self.views, self.pi_ts, self.nd, out=self.tm)
        sta.slack(self.g, self.views, self.nd, self.tm, self.ep_rat, out=self.sl)
        self.run += 1
        return self.run


class TNS(torch.autograd.Function):
    @staticmethod
    def forward(ctx, net_delay, load, td: TimedDesign):
        ctx.run = td.evaluate(net_delay, load)
        ctx.td = td
        ctx.save_for_backward(net_delay, load)
        return td.sl["tns"].clone()

    @staticmethod
    def backward(ctx, grad_tns):
        td = ctx.td
        if td.run != ctx.run:
            # the design's buffers were overwritten by a later forward pass: restore this
            # pass's argmax and slack state from its own inputs before the adjoint
            net_delay, load = ctx.saved_tensors
            ctx.run = td.evaluate(net_delay, load)
        adj = sta.tns_adjoint(td.g, td.lib, td.views, td.nd, td.tm, td.sl, out=td.adj)
        w = grad_tns.to(torch.float32)
        A = td.g.sizes["n_arcs"]
        D = td.g.sizes["n_drivers"]
        g_nd = (adj["g_net_delay"][:A] * w).sum(dim=1)
        g_load = (adj["g_load"][:D] * w).sum(dim=1)
        return g_nd, g_load, None


def tns(net_delay, load, td: TimedDesign):
    """TNS per view (FP64 tensor); differentiable in net_delay [A] and load [D]."""
    return TNS.apply(net_delay, load, td)
