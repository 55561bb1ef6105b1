"""FP64 reference of the learned part -- TEST INFRASTRUCTURE ONLY.

Follows the paper's Sec. II.B (training data and MLP): the network input is
{T, p, F(Y)} with F the Box-Cox transform (Eq. 7, lambda = 0.1), the output is
the change of the mass fractions over the step, u* = Y(t+dt) - Y(t), hidden
layers use GELU and the parameters are fitted with Adam on the data loss
(Eq. 8).  Readings where the text is silent or garbled:

* Eq. 7 prints x^{lambda-1}/lambda; the stated mapping of [0, 1] onto
  [-1/lambda, 0] fixes it as (x^lambda - 1)/lambda (log x when lambda = 0);
  negative mass fractions (integration round-off) are clamped to 0 first.
* Inputs and outputs are z-scored per feature with training-split statistics
  (sigma floored at 1e-12).
* GELU is the exact x Phi(x) form.
* Operands are rounded to bfloat16 (round-to-nearest-even) exactly where the
  GPU rounds them: weights, the network input and every hidden activation;
  the backward pass rounds the output gradient and every pre-activation
  gradient.  Sums are accumulated in float64 here.
* Adam follows Kingma & Ba (2015), Algorithm 1.
* The per-species networks (one network per mass fraction) each take the full
  input and give one output; a one-output network is trained as a K-output
  network whose data loss weights only its species' column.
* The physics losses (Eqs. 9-11) act on the z-scored outputs: Eq. 9 as the
  mean absolute deviation of the predicted mass fractions' sum from one,
  divided by the summed spread of dY; Eq. 10 on the heat release over the
  step, -(rho/dt) sum_k h_k(T) dY_k, divided by the RMS of the labels'.
"""
from __future__ import annotations

import numpy as np
from scipy.special import erf

LAMBDA = 0.1
SQRT2 = np.sqrt(2.0)


# ----------------------------------------------------------------------------
# transforms
# ----------------------------------------------------------------------------
def box_cox(x, lam=LAMBDA):
    """Eq. 7 (reading above): (x^lam - 1)/lam, or log x for lam = 0."""
    x = np.maximum(np.asarray(x, np.float64), 0.0)
    if lam == 0.0:
        return np.log(x)
    return (np.power(x, lam) - 1.0) / lam


def gelu(x):
    """x Phi(x) with Phi the standard normal CDF."""
    return 0.5 * x * (1.0 + erf(x / SQRT2))


def gelu_grad(x):
    """d/dx [x Phi(x)] = Phi(x) + x phi(x)."""
    return 0.5 * (1.0 + erf(x / SQRT2)) + x * np.exp(-0.5 * x * x) / np.sqrt(2.0 * np.pi)


def bf16(x):
    """Round to the nearest bfloat16 (ties to even) via float32; returns float64.

    float64 -> float32 first (as the GPU holds float32 values), then the 16
    low bits of the float32 pattern are rounded away."""
    f = np.asarray(x, np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    u = (u + 0x7FFF + lsb) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def f32(x):
    return np.asarray(x, np.float64).astype(np.float32).astype(np.float64)


# ----------------------------------------------------------------------------
# features and normalisation
# ----------------------------------------------------------------------------
def raw_features(T, p, Y):
    """[F(Y_1..Y_K), T, p] per cell (input set of Sec. II.B)."""
    return np.concatenate([box_cox(Y), np.asarray(T, np.float64)[:, None],
                           np.asarray(p, np.float64)[:, None]], axis=1)


def norm_stats(X, floor=1e-12):
    mu = X.mean(0)
    sd = np.maximum(X.std(0), floor)
    return mu, sd


# ----------------------------------------------------------------------------
# the network
# ----------------------------------------------------------------------------
def init_params(dims, seed):
    """He-uniform weights (U[-sqrt(6/fan_in), +]), zero biases.  W[l] is (in, out)."""
    rng = np.random.default_rng(seed)
    Ws, bs = [], []
    for i in range(len(dims) - 1):
        lim = np.sqrt(6.0 / dims[i])
        Ws.append(f32(rng.uniform(-lim, lim, (dims[i], dims[i + 1]))))
        bs.append(np.zeros(dims[i + 1]))
    return Ws, bs


def forward(Ws, bs, X, quantize=True):
    """MLP forward.  Returns (output, cache).  With ``quantize`` the operands
    are bfloat16-rounded where the GPU rounds them (see module docstring)."""
    q = bf16 if quantize else (lambda a: a)
    a = q(X)
    cache = {"A": [a], "Z": []}
    L = len(Ws)
    for i in range(L):
        z = a @ q(Ws[i]) + bs[i]
        if quantize:
            z = f32(z)
        cache["Z"].append(z)
        if i < L - 1:
            a = q(gelu(z))
            cache["A"].append(a)
        else:
            a = z
    return a, cache


def species_forward(nets, X, quantize=True):
    """Forward of the per-species networks (Sec. II.B: one network per
    species' mass fraction): nets[k] = (Ws, bs) of a network with one output;
    column k of the result [n, K] is network k's output."""
    return np.stack([forward(Ws, bs, X, quantize)[0][:, 0] for Ws, bs in nets], axis=1)


def species_split(Ws, bs):
    """The K one-output networks whose outputs are the columns of the K-output
    network (Ws, bs): network k keeps every hidden layer and column k of the
    output layer."""
    K = Ws[-1].shape[1]
    return [(list(Ws[:-1]) + [Ws[-1][:, k:k + 1]], list(bs[:-1]) + [bs[-1][k:k + 1]]) for k in range(K)]


def mse_loss(out, target):
    """Eq. 8 on normalised outputs: mean over samples and outputs."""
    d = out - target
    return float(np.mean(d * d)), 2.0 * d / d.size


def hrr_label_weights(species_thermo, W_g, T, p, Y, Y_next, dt, sd_y, scale=None):
    """Heat-release loss of Sec. II.B (Eq. 10), in the form the training uses.

    HRR = -(rho / dt) sum_k h_k(T) dY_k over the step, h_k the enthalpy per
    unit mass of species k at the input T [J/kg] (NASA-7: (h/RT) R_u T / W_k),
    rho = p Wbar / (R_u T) the input density [kg/m^3], dY = Y_next - Y the DI
    label.  Returns (G, s, hrr): G_ik = -(rho_i/dt) h_k(T_i) sd_k / s, the
    scale s (RMS of the label HRR over the rows unless given) and the label
    HRR itself.  species_thermo(T) -> (cp/R, h/RT, s/R) per species."""
    RU = 8.31446261815324
    T = np.asarray(T, np.float64)
    n, K = np.asarray(Y).shape
    Wkg = np.asarray(W_g, np.float64) * 1e-3
    h = np.empty((n, K))
    for i in range(n):
        _, hRT, _ = species_thermo(T[i])
        h[i] = np.asarray(hRT) * RU * T[i] / Wkg
    Y = np.asarray(Y, np.float64)
    Wbar = 1.0 / (Y / Wkg[None, :]).sum(1)
    rho = np.asarray(p, np.float64) * Wbar / (RU * T)
    hrr = -(rho / dt) * (h * (np.asarray(Y_next, np.float64) - Y)).sum(1)
    if scale is None:
        scale = float(np.sqrt(np.mean(hrr * hrr)))
    G = -(rho / dt)[:, None] * h * np.asarray(sd_y, np.float64)[None, :] / scale
    return G, scale, hrr


def phys_loss(out, target, mu_y, sd_y, G, w_mass, w_hrr, out_w=None):
    """Eq. 11 with W1 = 1 on z-scored outputs: the data loss of Eq. 8 plus
    w_mass times Eq. 9 and w_hrr times Eq. 10, and d(loss)/d(out).

    out_w [K] (optional) weights the data loss per output:
    sum_ik w_k d_ik^2 / (B sum_k w_k), the plain mean when all w_k are equal; a
    one-hot out_w is the loss of a network trained for one species alone (the
    per-species ensemble of Sec. II.B).

    Eq. 9: the predicted Y(t+dt) = Y + mu + sd out sums to one plus
    m_i = sum_k (mu_k + sd_k out_ik) (the inputs sum to one); the term is
    mean_i |m_i| / sum_k sd_k (scaled by the spread of dY so that it is of the
    order of the data loss).  Eq. 10: e_i = sum_k G_ik (out_ik - target_ik) is
    (HRR* - HRR) / s (hrr_label_weights); the term is mean_i e_i^2."""
    out = np.asarray(out, np.float64)
    target = np.asarray(target, np.float64)
    B = out.shape[0]
    d = out - target
    if out_w is None:
        loss = float(np.mean(d * d))
        grad = 2.0 * d / d.size
    else:
        w = np.asarray(out_w, np.float64)
        loss = float((w[None, :] * d * d).sum() / (B * w.sum()))
        grad = 2.0 * w[None, :] * d / (B * w.sum())
    mu_y = np.asarray(mu_y, np.float64)
    sd_y = np.asarray(sd_y, np.float64)
    if w_mass:
        m = (mu_y[None, :] + sd_y[None, :] * out).sum(1)
        S = sd_y.sum()
        loss += w_mass * float(np.mean(np.abs(m))) / S
        grad = grad + w_mass * np.sign(m)[:, None] * sd_y[None, :] / (S * B)
    if w_hrr:
        e = (np.asarray(G, np.float64) * d).sum(1)
        loss += w_hrr * float(np.mean(e * e))
        grad = grad + w_hrr * 2.0 * e[:, None] * np.asarray(G, np.float64) / B
    return loss, grad


def backward(Ws, bs, cache, dout, quantize=True):
    """Gradients of the loss w.r.t. W[l] (in, out) and b[l]."""
    q = bf16 if quantize else (lambda a: a)
    L = len(Ws)
    gW = [None] * L
    gb = [None] * L
    dz = q(dout)
    for i in range(L - 1, -1, -1):
        a = cache["A"][i]
        gW[i] = a.T @ dz
        gb[i] = dz.sum(0)
        if i > 0:
            da = dz @ q(Ws[i]).T
            dz = q(da * gelu_grad(cache["Z"][i - 1]))
    return gW, gb


def adam_step(p, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba 2015, Alg. 1).  Returns (p, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


# ----------------------------------------------------------------------------
# output side
# ----------------------------------------------------------------------------
def element_matrix(composition, element_mass):
    """E[e, k] = n_ek A_e / W_k: element e's mass fraction carried by species k."""
    comp = np.asarray(composition, np.float64)
    W = comp @ np.asarray(element_mass, np.float64)
    return (comp * np.asarray(element_mass)[None, :]).T / W[None, :]


def project_delta(Emat, Y, dY, floor=1e-30):
    """Element-conserving correction of dY (weights w_k = max(Y_k + dY_k, floor)):
    dY <- dY - w E^T (E w E^T)^-1 E dY, so that E dY = 0."""
    out = np.empty_like(dY)
    for c in range(dY.shape[0]):
        w = np.maximum(Y[c] + dY[c], floor)
        A = (Emat * w[None, :]) @ Emat.T
        lam = np.linalg.solve(A, Emat @ dY[c])
        out[c] = dY[c] - w * (Emat.T @ lam)
    return out


def project_weighted(Emat, target, y, w):
    """The vector closest to y in the weighted norm sum_k (y'_k - y_k)^2 / w_k
    whose element masses Emat y' equal `target`; species with w_k = 0 are held
    where they are.  Lagrange's condition gives
        y' = y - W E^T (E W E^T)^-1 (E y - target),   W = diag(w).
    Returns (y', ok), ok False when E W E^T is singular (an element carried
    only by held species cannot be restored)."""
    A = (Emat * w[None, :]) @ Emat.T
    try:
        lam = np.linalg.solve(A, Emat @ y - target)
    except np.linalg.LinAlgError:
        return y.copy(), False
    return y - w * (Emat.T @ lam), True


POST_ROUNDS = 4


def post_state(Emat, Y, dY, sd, rounds=POST_ROUNDS, neg_tol=1e-6):
    """State after the network's step (the post-processing of the chemistry
    advance with the learned source term), per cell:

    * the prediction y* = Y + dY is corrected to the nearest state with the
      input's element masses E Y, nearness measured in units of each
      species' spread sd_k of dY in the training data (weights w_k = sd_k^2:
      the network is fitted on dY / sd, so its errors are of similar size in
      those units for every species);
    * species the correction leaves negative are held at zero and the
      correction is solved again from y* over the remaining species, at most
      `rounds` solves in all.

    Returns (Y_new, ok, adj): ok is False when a solve is singular, the
    result is not finite or some Y_k stays below -neg_tol (such cells are
    advanced by DI); adj = max_k |Y_new,k - y*_k| / sd_k is the size of the
    whole correction in those units."""
    n, K = Y.shape
    sd = np.asarray(sd, np.float64)
    out = np.empty_like(Y)
    ok = np.ones(n, bool)
    adj = np.zeros(n)
    for c in range(n):
        ystar = Y[c] + dY[c]
        target = Emat @ Y[c]
        held = np.zeros(K, bool)
        for _ in range(rounds):
            y1 = np.where(held, 0.0, ystar)
            w = np.where(held, 0.0, sd * sd)
            y2, good = project_weighted(Emat, target, y1, w)
            if not good:
                ok[c] = False
                break
            neg = ~held & (y2 < 0.0)
            if not neg.any():
                break
            held |= neg
        out[c] = y2
        ok[c] = ok[c] and bool(np.all(np.isfinite(y2))) and y2.min() >= -neg_tol
        adj[c] = np.max(np.abs(y2 - ystar) / sd)
    return out, ok, adj
