"""Backward-Euler absorption/emission/scattering split (paper Sec. 3.2).

Eq. couple_a solved for I^{m+1} gives
    I^{m+1} = d (I* + c dt rho kappa_s J^{m+1} + c dt rho kappa_a (c / 4 pi) a_r T_dag^4),
    d = 1 / (1 + c dt rho (kappa_a + kappa_s)),
where I* is the post-transport intensity (operator splitting).  Integrating
over solid angle (J = (1/4pi) sum I dOmega = (c/4pi) E) and solving for the
new mean intensity,
    J^{m+1} = (J* + c dt rho kappa_a (c / 4 pi) a_r T_dag^4) / (1 + c dt rho kappa_a),
which does not involve kappa_s (isotropic scattering moves no energy
between the radiation and the material).  Inserting it into eq. couple_b
gives the scalar equation
    f(T) = T - T^m + (c dt kappa_a / c_v) (a_r T^4 - E*) / (1 + c dt rho kappa_a) = 0
("a simple fourth order polynomial root find").  f is increasing and convex
for T > 0, so the positive root is unique and Newton's method started at
T0 = max(T^m, (max(E*,0)/a_r)^(1/4)), where f(T0) >= 0, decreases
monotonically onto it.  Stopping rule: |dT| <= 4 u T, at most 50 iterations.

The isotropic source added to the intensity is then the rank-1 tensor
s (x) 1 (x) 1 with s = d (c dt rho kappa_s J^{m+1} + c dt rho kappa_a (c/4pi)
a_r T_dag^4) (Sec. 4.4); without scattering s = d c dt rho kappa_a (c/4pi)
a_r T_dag^4.

Temperature update (energy-conserving form stated at the end of Sec. 3.2):
    rho c_v (T^{m+1} - T^m) = E* - E^{m+1},
reading the paper's J^m as the post-transport mean intensity (the state the
source substep starts from) and E^{m+1} as the energy of the final
(rounded) intensity.  In frozen mode T never changes.
"""
import numpy as np

U = 2.0 ** -53


def newton_temperature(Estar, Tm, kappa, rho, cv, c, dt, a_r, max_iter=50):
    """Solve f(T) = 0 per cell (vectorised); returns (T_dag, converged)."""
    Estar = np.asarray(Estar, float)
    Tm = np.asarray(Tm, float)
    g = c * dt * kappa / cv / (1.0 + c * dt * rho * kappa)
    T = np.maximum(Tm, (np.maximum(Estar, 0.0) / a_r) ** 0.25)
    done = np.zeros(T.shape, bool)
    for _ in range(max_iter):
        f = T - Tm + g * (a_r * T ** 4 - Estar)
        fp = 1.0 + 4.0 * g * a_r * T ** 3
        dT = f / fp
        Tn = np.where(done, T, T - dT)
        done |= np.abs(dT) <= 4 * U * np.abs(T)
        T = Tn
        if done.all():
            break
    return T, bool(done.all())


def source_coefficients(Estar, T, setup):
    """Return (d, s, T_dag) per cell for the step starting at temperature T.

    ``Estar`` is the energy density of the post-transport intensity; it
    enters through the Newton solve (coupled material) and through
    J^{m+1} (scattering)."""
    c, dt, a_r = setup.c, setup.dt, setup.a_r
    rk = setup.rho * setup.kappa
    rs = setup.rho * setup.kappa_s
    d = 1.0 / (1.0 + c * dt * (rk + rs))
    if setup.material == 1:
        Tdag, ok = newton_temperature(Estar, T, setup.kappa, setup.rho,
                                      setup.cv, c, dt, a_r)
        if not ok:
            raise FloatingPointError("Newton did not converge")
    else:
        Tdag = T.copy()
    emis = c * dt * rk * (c / (4.0 * np.pi)) * a_r * Tdag ** 4
    s = d * emis
    if setup.scatter:
        Jstar = c / (4.0 * np.pi) * np.asarray(Estar, float)
        Jnew = (Jstar + emis) / (1.0 + c * dt * rk)
        s = d * (c * dt * rs * Jnew + emis)
    return d, s, Tdag


def temperature_update(T, Estar, Enew, setup):
    if setup.material != 1:
        return T.copy()
    return T + (Estar - Enew) / (setup.rho * setup.cv)
