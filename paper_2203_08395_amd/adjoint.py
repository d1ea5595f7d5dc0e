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


class TNS(torch.autograd.Function):
    @staticmethod
    def forward(ctx, net_delay, load, td: TimedDesign):
        td.nd["net_delay"].copy_(net_delay)
        td.nd["load"].copy_(load)
        sta.arc_load(td.g, td.nd)
        sta.propagate(td.g, td.lib, td.views, td.pi_ts, td.nd, out=td.tm)
        sta.slack(td.g, td.views, td.nd, td.tm, td.ep_rat, out=td.sl)
        ctx.td = td
        return td.sl["tns"].clone()

    @staticmethod
    def backward(ctx, grad_tns):
        td = ctx.td
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
