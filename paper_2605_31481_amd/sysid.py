"""Identification of link masses by gradient descent through RNEA (Sec. 4.3).

The masses are the unknowns; every other inertial property of a link keeps
its nominal value in the frame of its centre of mass (the COM position c and
the rotational inertia I_C about the COM), and the body-origin parameters the
model uses, [m, m c, I_C + m (|c|^2 1 - c c^T)], are rebuilt from the masses
at every evaluation.  That map is affine in the masses, pi(m) = A + m D per
link, so the gradient of a loss with respect to the masses is the gradient
with respect to the inertial parameters contracted with D.

The loss is the mean squared torque residual over a batch of measured states,
    L(m) = 1/(2B) sum_b |RNEA(q_b, qd_b, qdd_b; pi(m)) - tau_b|^2,
evaluated with one RNEA launch, and its parameter gradient with one RNEA
adjoint launch whose cotangent is the residual over B (the batch sum of the
inertial-parameter gradient is reduced on the device).  The optimiser is
PyTorch's L-BFGS over the n link masses; all per-instance work runs in the
library's kernels.

Because pi is affine in m and RNEA is linear in pi, L is a quadratic in m
with Hessian H = Phi^T Phi / B, Phi_k = RNEA(q, qd, qdd; D_k) the torques of
link k's mass direction alone.  Link masses excite the torques very unevenly
(a distal link's column is far smaller than a base link's), so H is badly
scaled; L-BFGS runs on u = m / s with s_k = 1 / sqrt(H_kk), the diagonal
(Jacobi) scaling, whose n columns cost n RNEA launches once per problem.
"""

from __future__ import annotations

import numpy as np

from . import bard


def mass_map(inertia) -> tuple:
    """Split body-origin parameters [n, 10] (m, m c, I_O as xx, xy, yy, xz,
    yz, zz) into pi(m) = A + m D with the COM and the rotational inertia about
    the COM held fixed.  Returns (A, D, m), FP64."""
    pi = np.asarray(inertia, dtype=np.float64).reshape(-1, 10)
    m = pi[:, 0].copy()
    if np.any(m <= 0):
        raise ValueError("every link needs a positive nominal mass")
    c = pi[:, 1:4] / m[:, None]
    cx, cy, cz = c[:, 0], c[:, 1], c[:, 2]
    D = np.zeros_like(pi)
    D[:, 0] = 1.0
    D[:, 1:4] = c
    D[:, 4] = cy * cy + cz * cz
    D[:, 5] = -cx * cy
    D[:, 6] = cx * cx + cz * cz
    D[:, 7] = -cx * cz
    D[:, 8] = -cy * cz
    D[:, 9] = cx * cx + cy * cy
    A = pi - m[:, None] * D
    return A, D, m


class MassIdentification:
    """Least-squares mass identification on one batch of measurements.

    q, qd, qdd, tau_meas: device tensors [K, B] (instance-minor, the layout of
    the operators) of one dtype; inertia: the nominal [n, 10] parameters whose
    COM and rotational inertia are kept."""

    def __init__(self, model: bard.Model, inertia, q, qd, qdd, tau_meas, precondition: bool = True):
        torch = bard._torch()
        A, D, m = mass_map(inertia)
        self.model = model
        self.dtype, self.device = q.dtype, q.device
        self.A = torch.tensor(A, dtype=self.dtype, device=self.device)
        self.D = torch.tensor(D, dtype=self.dtype, device=self.device)
        self.m_nominal = m
        self.q, self.qd, self.qdd, self.tau_meas = q, qd, qdd, tau_meas
        self.B = int(q.shape[1])
        self.evaluations = 0
        self.scale = self.jacobi_scale() if precondition else np.ones(len(m))

    def jacobi_scale(self) -> np.ndarray:
        """s_k = 1 / sqrt(H_kk), H_kk = |RNEA(q, qd, qdd; D_k)|^2 / B: one RNEA
        launch per link with that link's mass direction as its only
        parameters."""
        torch = bard._torch()
        n = self.D.shape[0]
        s = np.ones(n)
        for k in range(n):
            pi = torch.zeros_like(self.D)
            pi[k] = self.D[k]
            t = self.model.rnea(self.q, self.qd, self.qdd, inertia=pi)
            h = float((t.double() * t.double()).sum()) / self.B
            s[k] = 1.0 / np.sqrt(h) if h > 0 else 1.0
        return s

    def inertia(self, m):
        """Body-origin parameters [n, 10] for the masses m (device tensor [n])."""
        return (self.A + m[:, None] * self.D).contiguous()

    def loss_and_grad(self, m):
        """(L(m), dL/dm) for masses m, a device tensor [n] of the batch dtype."""
        pi = self.inertia(m)
        tau = self.model.rnea(self.q, self.qd, self.qdd, inertia=pi)
        r = (tau - self.tau_meas) * (1.0 / self.B)
        loss = 0.5 * self.B * (r * r).sum()
        _, _, _, pib = self.model.rnea_vjp(self.q, self.qd, self.qdd, r.contiguous(), inertia=pi)
        self.evaluations += 1
        return loss, (pib * self.D).sum(dim=1)

    def run(self, m0, max_iter: int = 20, history: int = 10, tolerance_grad: float = 1e-9,
            tolerance_change: float = 1e-12) -> dict:
        """L-BFGS (strong Wolfe line search) from masses m0; returns the
        identified masses, the final loss, the iterations and the number of
        loss/gradient evaluations."""
        torch = bard._torch()
        # the optimiser works on u = m / s and keeps its state in FP64;
        # evaluations run in the batch dtype
        s = torch.tensor(self.scale, dtype=torch.float64, device=self.device)
        u = torch.nn.Parameter(torch.tensor(np.asarray(m0, dtype=np.float64), dtype=torch.float64,
                                            device=self.device) / s)
        opt = torch.optim.LBFGS([u], lr=1.0, max_iter=max_iter, history_size=history,
                                line_search_fn="strong_wolfe", tolerance_grad=tolerance_grad,
                                tolerance_change=tolerance_change)
        e0 = self.evaluations

        def closure():
            loss, g = self.loss_and_grad((u.detach() * s).to(self.dtype))
            u.grad = g.to(torch.float64) * s
            return loss.to(torch.float64)

        opt.step(closure)
        state = opt.state[opt._params[0]]
        m = (u.detach() * s)
        loss, _ = self.loss_and_grad(m.to(self.dtype))
        return {"masses": m.cpu().numpy(), "loss": float(loss),
                "iterations": int(state.get("n_iter", 0)), "evaluations": self.evaluations - e0}


def noisy_torques(tau_true, fraction: float, seed: int):
    """tau_true plus independent Gaussian noise per joint with standard
    deviation fraction x the joint's RMS torque over the batch ([K, B] device
    tensor in, same out)."""
    torch = bard._torch()
    g = torch.Generator(device=tau_true.device)
    g.manual_seed(int(seed))
    rms = tau_true.pow(2).mean(dim=1, keepdim=True).sqrt()
    noise = torch.randn(tau_true.shape, generator=g, device=tau_true.device, dtype=tau_true.dtype)
    return tau_true + fraction * rms * noise


def perturbed_masses(m_true, fraction: float, seed: int) -> np.ndarray:
    """Each mass scaled by 1 + fraction or 1 - fraction, the sign drawn per
    link."""
    rng = np.random.default_rng(seed)
    return np.asarray(m_true) * (1.0 + fraction * rng.choice([-1.0, 1.0], size=len(m_true)))


def identify(model: bard.Model, inertia_true, q, qd, qdd, seeds=range(10), perturbation: float = 0.3,
             noise: float = 0.05, max_iter: int = 20, tau_true=None, precondition: bool = True) -> dict:
    """The identification experiment: torques from the true parameters
    (computed by the library unless tau_true is given) plus `noise` x RMS
    Gaussian noise per joint, masses started `perturbation` away from the
    truth with random signs, one L-BFGS run per seed.  Returns per-seed
    identified masses and relative errors."""
    torch = bard._torch()
    pi_true = torch.tensor(np.asarray(inertia_true, dtype=np.float64), dtype=q.dtype, device=q.device).contiguous()
    if tau_true is None:
        tau_true = model.rnea(q, qd, qdd, inertia=pi_true)
    _, _, m_true = mass_map(inertia_true)
    out = {"m_true": m_true, "masses": [], "rel_error": [], "iterations": [], "evaluations": []}
    for s in seeds:
        tau_meas = noisy_torques(tau_true, noise, 7000 + s) if noise > 0 else tau_true
        prob = MassIdentification(model, inertia_true, q, qd, qdd, tau_meas, precondition=precondition)
        res = prob.run(perturbed_masses(m_true, perturbation, 8000 + s), max_iter=max_iter)
        out["masses"].append(res["masses"])
        out["rel_error"].append(np.abs(res["masses"] - m_true) / m_true)
        out["iterations"].append(res["iterations"])
        out["evaluations"].append(res["evaluations"])
    for k in ("masses", "rel_error"):
        out[k] = np.asarray(out[k])
    return out
