"""Oracle-side transport coefficients of the reduced model (TEST INFRASTRUCTURE).

Written from the Chapman-Enskog results of Sec. 4 (hydrodynamics):
  gamma  = (5 + delta)/(3 + delta)
  eta    = p tau/(B - b),   B = 1 + tau/tau1
  eta_b  = 2 delta p tau1 / (3 (3 + delta))
  kappa  = 5 p tau (1 + k_r)/(2 B),   k_r = kappa_R/kappa_T
  Pr     = (B/(B - b)) (1 + delta/5)/(1 + k_r)
and the Landau number of Sec. 6 (sound absorption):
  La = Kn (4/3 + eta_b/eta) + Kn (gamma - 1)/Pr.
Kept separate from the product's parameter resolver on purpose.
"""
import math

THETA0 = 0.2948964908710633


def coefficients(tau, tau1, b, kr, delta, theta0=THETA0, rho=1.0):
    """Macroscopic coefficients implied by (tau, tau1, b, k_r, delta)."""
    B = 1.0 + tau / tau1
    p = rho * theta0
    eta = p * tau / (B - b)
    eta_b = 2.0 * delta * p * tau1 / (3.0 * (3.0 + delta))
    kappa_T = 5.0 * p * tau / (2.0 * B)
    kappa = kappa_T * (1.0 + kr)
    gamma = (5.0 + delta) / (3.0 + delta)
    cp = (5.0 + delta) / 2.0
    Pr = (B / (B - b)) * (1.0 + delta / 5.0) / (1.0 + kr)
    nu = eta / rho
    return dict(B=B, eta=eta, eta_b=eta_b, nu=nu, nu_b=eta_b / rho, kappa=kappa,
                kappa_T=kappa_T, kappa_R=kr * kappa_T, gamma=gamma, cp=cp, Pr=Pr,
                alpha=kappa / (rho * cp), cs=math.sqrt(gamma * theta0),
                lam_b=eta_b / eta)


def resolve(nu, Pr, lam_b, delta, theta0=THETA0, b=None, kr=None):
    """(nu, Pr, eta_b/eta, delta) -> (tau, tau1, b, k_r).

    The map has one free direction.  Rule: start from k_r = delta/5; solve b
    from Pr; clamp b to the ES range [-1/2, 1]; then tau1/tau from eta_b/eta,
    k_r from Pr, tau from nu.  An explicit b (or k_r) replaces that step.  An
    explicit b may exceed 1 (Sec. 6 runs its Landau-number table at Pr 5 and
    10 with tau = 3 tau1/5 and k_r = 0, which needs b = 1.152 and 1.376); it
    must stay below B = 1 + tau/tau1, where the shear viscosity p tau/(B - b)
    is positive.
    """
    cd = 2.0 * delta / (3.0 * (3.0 + delta))
    if b is None:
        if kr is None:
            kr = delta / 5.0
        # with B/(B-b) = Pr (1+k_r)/(1+delta/5) =: P and lam_b = cd (tau1 + tau (1-b) ... )
        P = Pr * (1.0 + kr) / (1.0 + delta / 5.0)
        # B - b = B/P ; lam_b = cd tau1 (B - b)/tau = cd (tau1 + tau)/(tau P)
        r = lam_b * P / cd - 1.0           # tau1/tau
        if r <= 0:
            raise ValueError("infeasible")
        B = 1.0 + 1.0 / r
        b = B * (1.0 - 1.0 / P)
        b = min(max(b, -0.5), 1.0)
    if b == 1.0:
        raise ValueError("b = 1 needs an explicit tau1")
    if b < -0.5:
        raise ValueError("b below the ES range")
    r = (lam_b / cd - 1.0) / (1.0 - b)      # tau1/tau from lam_b = cd (1 + (1-b) tau1/tau)
    if not r > 0:
        raise ValueError("infeasible: no positive tau1/tau gives this eta_b/eta "
                         "(b < 1 needs it above 2 delta/(3(3+delta)), b > 1 below)")
    B = 1.0 + 1.0 / r
    if not b < B:
        raise ValueError("infeasible: b >= 1 + tau/tau1 (no positive shear viscosity)")
    kr_new = (B / (B - b)) * (1.0 + delta / 5.0) / Pr - 1.0
    if kr_new < -1e-12:
        raise ValueError("infeasible: k_r < 0")
    kr = max(kr_new, 0.0)
    tau = nu * (B - b) / theta0
    tau1 = r * tau
    return dict(tau=tau, tau1=tau1, b=b, kr=kr, delta=delta)
