"""EnSF analysis step in FP64 (oracle; test infrastructure only).

Follows Sec. III-A of the paper.  Notation: X (N x d) is the forecast (prior) ensemble,
Z (P x d) the particles pushed through the reverse-time SDE, t in (0, 1] pseudo-time.

Readings taken where the paper is silent or garbled:
  * schedule alpha_t = 1 - t(1 - eps), beta_t^2 = t, eps = 0.05 (eq. 9 with the
    printed alpha_t = 1 - t is singular at t = 1);
  * b = d log(alpha)/dt and sigma^2 = d(beta^2)/dt - 2 b beta^2, eq. 9;
  * damping h(t) = 1 - t (eq. 11 with T = 1);
  * the weights of eq. 16 normalise Q(z | x_j) over the forecast members x_j;
  * the likelihood is the Gaussian of eq. 5 with the conventional 1/2,
    log p(y | z) = -sum_m (y_m - g(z_{idx_m}))^2 / (2 sigma_o^2), g = arctan or identity;
  * uniform pseudo-time grid dt = 1/K, the score evaluated at t_k = 1 - k dt for
    k = 0 .. K-1, and plain Euler-Maruyama with noise on every step (eq. 7):
        z <- z - (b z - sigma^2 s) dt + sqrt(sigma^2 dt) xi.
"""
import numpy as np

from . import philox


def schedule(t, eps=0.05):
    """Drift and diffusion coefficients of the forward SDE (eq. 6, eq. 9) and the damping
    weight h(t) (eq. 11) at pseudo-time t."""
    t = float(t)
    alpha = 1.0 - t * (1.0 - eps)
    beta2 = t
    b = -(1.0 - eps) / alpha                       # d/dt log(alpha_t)
    sigma2 = 1.0 - 2.0 * b * beta2                 # d(beta^2)/dt - 2 b beta^2
    h = 1.0 - t
    return dict(alpha=alpha, beta2=beta2, b=b, sigma2=sigma2, h=h)


def densify(obs_idx, obs_val, d, sigma_o):
    """Per-component sums of the Gaussian likelihood (eq. 2, eq. 5 with R = sigma_o^2 I):
    A[e] = sum_{m: idx_m = e} y_m / sigma_o^2,  B[e] = #{m: idx_m = e} / sigma_o^2."""
    A = np.zeros(d)
    B = np.zeros(d)
    idx = np.asarray(obs_idx, dtype=np.int64)
    np.add.at(A, idx, np.asarray(obs_val, dtype=np.float64) / sigma_o ** 2)
    np.add.at(B, idx, 1.0 / sigma_o ** 2)
    return A, B


def log_likelihood(z, obs_idx, obs_val, sigma_o, obs_op="arctan"):
    """log p(y | z) up to a constant, for one state vector z."""
    g = np.arctan(z[obs_idx]) if obs_op == "arctan" else z[obs_idx]
    r = np.asarray(obs_val, dtype=np.float64) - g
    return -0.5 * np.sum(r * r) / sigma_o ** 2


def likelihood_score(Z, A, B, obs_op="arctan"):
    """Gradient of log p(y | z) for every particle row of Z, from the densified sums."""
    if obs_op == "arctan":
        return (A - B * np.arctan(Z)) / (1.0 + Z * Z)
    return A - B * Z


def likelihood_curvature(Z, B, obs_op="arctan"):
    """Gauss-Newton curvature of -log p(y | z) per component: B * g'(z)^2 with g the
    observation operator (g' = 1 for the identity, 1 / (1 + z^2) for arctan).  It is the
    stiffness of the likelihood term that the linearly implicit step treats implicitly."""
    if obs_op == "arctan":
        return B / (1.0 + Z * Z) ** 2
    return B * np.ones_like(Z)


def prior_weights(Z, X, t, eps=0.05):
    """Monte-Carlo weights of eq. 16: w_ij = Q(z_i | x_j) / sum_j' Q(z_i | x_j'), with
    Q(z | x) proportional to exp(-|z - alpha x|^2 / (2 beta^2)) (eq. 12).
    The squared distance is expanded as |z|^2 - 2 alpha z.x + alpha^2 |x|^2; the row
    maximum is subtracted before exponentiating (it cancels in the ratio)."""
    s = schedule(t, eps)
    a, beta2 = s["alpha"], s["beta2"]
    G = Z @ X.T
    zz = np.sum(Z * Z, axis=1)
    xx = np.sum(X * X, axis=1)
    logq = -(zz[:, None] - 2.0 * a * G + a * a * xx[None, :]) / (2.0 * beta2)
    logq -= logq.max(axis=1, keepdims=True)
    q = np.exp(logq)
    return q / q.sum(axis=1, keepdims=True)


def prior_score(Z, X, t, eps=0.05, return_weights=False):
    """Monte-Carlo prior score of eq. 15 with the whole ensemble as the mini-batch:
    s(z_i) = sum_j -(z_i - alpha x_j) / beta^2 * w_ij."""
    s = schedule(t, eps)
    W = prior_weights(Z, X, t, eps)
    S = -(W.sum(axis=1, keepdims=True) * Z - s["alpha"] * (W @ X)) / s["beta2"]
    return (S, W) if return_weights else S


def prior_score_bruteforce(Z, X, t, eps=0.05):
    """The same score by explicit loops over particles, members and components (tiny
    inputs only; no expansion of the distance, no max subtraction)."""
    s = schedule(t, eps)
    a, beta2 = s["alpha"], s["beta2"]
    P, d = Z.shape
    N = X.shape[0]
    S = np.zeros((P, d))
    W = np.zeros((P, N))
    for i in range(P):
        q = []
        for j in range(N):
            dist = 0.0
            for e in range(d):
                diff = Z[i, e] - a * X[j, e]
                dist += diff * diff
            q.append(np.exp(-dist / (2.0 * beta2)))
        tot = sum(q)
        for j in range(N):
            W[i, j] = q[j] / tot
            for e in range(d):
                S[i, e] += -(Z[i, e] - a * X[j, e]) / beta2 * W[i, j]
    return S, W


def posterior_score(Z, X, A, B, t, eps=0.05, obs_op="arctan"):
    """Damped posterior score of eq. 11 / eq. 17: prior score + h(t) * likelihood score."""
    s = schedule(t, eps)
    return prior_score(Z, X, t, eps) + s["h"] * likelihood_score(Z, A, B, obs_op)


def initial_particles(seed, filter_id, particle_ids, d):
    """Z at t = 1: standard normal draws (Sec. III-A-2)."""
    return philox.normals(seed, filter_id, philox.INIT_STEP, particle_ids, d)


def analysis(X, obs_idx, obs_val, sigma_o, n_steps, seed, filter_id=0, obs_op="arctan",
             eps=0.05, n_particles=None, particle_ids=None, spread_relax=0.0, chunk=1024,
             return_all=False, lik_step="explicit"):
    """Analysis ensemble: run the discretised reverse SDE (eq. 7) from N(0, I) with the
    approximate posterior score (eq. 17).  Particles are independent given X, so any
    subset `particle_ids` of the n_particles particles can be run alone; `chunk` bounds
    the rows of the Gram matrix held at once.

    lik_step = "explicit" is the plain Euler-Maruyama step of eq. 7 (the paper's "e.g.,
    an Euler scheme").  lik_step = "implicit" advances the damped likelihood part of the
    drift, sigma^2 h s_lik(z), linearly implicitly with its Gauss-Newton curvature kappa:
        z <- z - (b z - sigma^2 s_prior) dt + sigma^2 h s_lik dt / (1 + sigma^2 h kappa dt)
               + sqrt(sigma^2 dt) xi,
    which equals the explicit step where there are no observations and stays stable when
    dt is not small against sigma_o^2 (the explicit step needs dt of order sigma_o^2)."""
    if lik_step not in ("explicit", "implicit"):
        raise ValueError(lik_step)
    X = np.asarray(X, dtype=np.float64)
    N, d = X.shape
    if particle_ids is None:
        particle_ids = np.arange(n_particles if n_particles is not None else N)
    particle_ids = np.asarray(particle_ids, dtype=np.int64)
    A, B = densify(obs_idx, obs_val, d, sigma_o)
    Z = initial_particles(seed, filter_id, particle_ids, d)
    dt = 1.0 / n_steps
    for k in range(n_steps):
        t = 1.0 - k * dt
        sc = schedule(t, eps)
        xi = philox.normals(seed, filter_id, k, particle_ids, d)
        for c0 in range(0, Z.shape[0], chunk):
            z = Z[c0:c0 + chunk]
            noise = np.sqrt(sc["sigma2"] * dt) * xi[c0:c0 + chunk]
            if lik_step == "explicit":
                S = posterior_score(z, X, A, B, t, eps, obs_op)
                Z[c0:c0 + chunk] = z - (sc["b"] * z - sc["sigma2"] * S) * dt + noise
            else:
                Sp = prior_score(z, X, t, eps)
                L = likelihood_score(z, A, B, obs_op)
                kap = likelihood_curvature(z, B, obs_op)
                damp = sc["sigma2"] * sc["h"] * dt
                Z[c0:c0 + chunk] = (z - (sc["b"] * z - sc["sigma2"] * Sp) * dt
                                    + damp * L / (1.0 + damp * kap) + noise)
    if spread_relax > 0.0:
        Z = relax_spread(Z, X, spread_relax)
    return Z


def relax_spread(Z, X, r):
    """Relaxation of the analysis spread toward the prior spread (Sec. IV-A), per
    component: z <- mean + (z - mean) * (1 - r + r * sd_prior / sd_post), ddof = 1."""
    mean = Z.mean(axis=0)
    sd_post = Z.std(axis=0, ddof=1)
    sd_prior = np.asarray(X, dtype=np.float64).std(axis=0, ddof=1)
    with np.errstate(divide="ignore", invalid="ignore"):
        fac = np.where(sd_post > 0, 1.0 - r + r * sd_prior / sd_post, 1.0)
    return mean + (Z - mean) * fac


def posterior_stats(Z):
    """Posterior mean and spread (per-component std, ddof = 1) over the particles."""
    return Z.mean(axis=0), Z.std(axis=0, ddof=1)


def rel_l2(a, b):
    """||a - b||_2 / ||b||_2 over all entries (b is the reference)."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))
