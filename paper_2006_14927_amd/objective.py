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
    mask = (S_target >= min_photons).to(S.dtype)
    rel = (S - S_target) / (S_target + count_floor)
    M = A / torch.where(S > 0, S, torch.ones_like(S))
    Mt = A_target / torch.where(S_target > 0, S_target, torch.ones_like(S_target))
    return (rel * rel).sum() + (mask * ((M - Mt) / time_scale_ns) ** 2).sum()
