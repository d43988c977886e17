"""Closed-form check of the Euler-Maruyama scheme for a Gaussian prior and a linear,
Gaussian observation (oracle; test infrastructure only).

If the prior of one component is N(mu, s2) and the prior score is the exact score of its
diffused law N(alpha mu, alpha^2 s2 + beta^2) (eq. 12 marginalised), the posterior score
of eq. 11 is affine in z, so one Euler-Maruyama step of eq. 7 maps the particle mean m
and variance v exactly:
    v_t = alpha^2 s2 + beta^2,   c = 1/v_t + h B,   q = alpha mu / v_t + h A,
    P   = 1 - b dt - sigma^2 c dt,
    m <- P m + sigma^2 q dt,     v <- P^2 v + sigma^2 dt,
starting from m = 0, v = 1 at t = 1, with A = y/sigma_o^2 and B = 1/sigma_o^2 for an
observed component (A = B = 0 otherwise).  The Monte-Carlo score of eq. 15 tends to the
exact score as the ensemble grows (in low dimension), so particle statistics of the full
scheme must approach (m, v).  The damped score does not reproduce the Kalman posterior;
`kalman` gives it for reporting the gap.
"""
from .ensf import schedule


def em_recursion(mu, s2, A, B, n_steps, eps=0.05, lik_step="explicit"):
    """lik_step = "implicit": the likelihood part of the drift, sigma^2 h (A - B z) dt, is
    divided by (1 + sigma^2 h B dt) (the identity operator's curvature is B), so
        P = 1 - b dt - sigma^2 dt / v_t - g B,   m <- P m + sigma^2 alpha mu dt / v_t + g A,
    with g = sigma^2 h dt / (1 + sigma^2 h B dt)."""
    m, v = 0.0, 1.0
    dt = 1.0 / n_steps
    for k in range(n_steps):
        t = 1.0 - k * dt
        sc = schedule(t, eps)
        vt = sc["alpha"] ** 2 * s2 + sc["beta2"]
        if lik_step == "explicit":
            c = 1.0 / vt + sc["h"] * B
            q = sc["alpha"] * mu / vt + sc["h"] * A
            P = 1.0 - sc["b"] * dt - sc["sigma2"] * c * dt
            m = P * m + sc["sigma2"] * q * dt
        else:
            g = sc["sigma2"] * sc["h"] * dt / (1.0 + sc["sigma2"] * sc["h"] * B * dt)
            P = 1.0 - sc["b"] * dt - sc["sigma2"] * dt / vt - g * B
            m = P * m + sc["sigma2"] * sc["alpha"] * mu * dt / vt + g * A
        v = P * P * v + sc["sigma2"] * dt
    return m, v


def kalman(mu, s2, y, sigma_o2):
    """Posterior mean and variance of N(mu, s2) observed once as y = x + N(0, sigma_o2)."""
    g = s2 / (s2 + sigma_o2)
    return mu + g * (y - mu), (1.0 - g) * s2
