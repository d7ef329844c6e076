"""Example objective on the soft telescope response (user-level code).

For each shower s and telescope k, with S* and A* the response of a target
atmosphere:
    L = sum_sk ((S - S*) / (S* + 10))^2 + [S* >= 100] ((A/S - A*/S*) / 1 ns)^2,
i.e. relative photon-count residuals plus mean-arrival-time residuals where the
target sees at least 100 photons.  It acts on (n_showers, n_tel) aggregates only;
the expensive part, (S, A) and their gradients, runs in the HIP library.
"""


def telescope_loss(S, A, S_target, A_target, count_floor=10.0, time_scale_ns=1.0,
                   min_photons=100.0):
    import torch
    rel = (S - S_target) / (S_target + count_floor)
    # mean times only where the target sees enough light; the divisions are
    # masked before they happen, so a tiny S elsewhere cannot turn the gradient
    # into 0 * inf
    use = (S_target >= min_photons) & (S > 0)
    one = torch.ones_like(S)
    M = A / torch.where(use, S, one)
    Mt = A_target / torch.where(use, S_target, one)
    dt = torch.where(use, (M - Mt) / time_scale_ns, torch.zeros_like(S))
    return (rel * rel).sum() + (dt * dt).sum()
