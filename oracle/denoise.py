"""Learned current denoiser: plain FP64 reference (test infrastructure only).

The method's current deposit is noisy at few particles per cell; the learned
part maps the raw deposit of a low-ppc run to a correction of the binomially
filtered current, trained against the filtered current of a high-ppc run.
Readings taken here (the paper has no learned part; its filter is the
1-2-1 pass of the field solver):

* Network: four 3x3x3 convolutions, channels 3 -> 16 -> 32 -> 16 -> 3, ReLU
  after the first three, "same" padding that is periodic in x and y (the
  transverse directions are periodic) and zero in zeta, no normalisation.
  Convolution is cross-correlation: y[o, v] = b[o] + sum_{c, t} W[o, c, t]
  x[c, v + off(t)], taps t = (kz, ky, kx) with offsets (kz - 1, ky - 1, kx - 1).
* Input: the raw deposited (J_x, J_y, J_z) divided by the electron density n_e.
* Output A lives on cell faces (A_x at (i, j+1/2, n+1/2), A_y at
  (i+1/2, j, n+1/2), A_z at (i+1/2, j+1/2, n)); the denoised current is
  J = F(J_raw) + s D x A with s = n_e h, F the binomial filter and D x the
  staggered curl whose differences match the deposit's staggering
  (J_x at (i+1/2, j, n), J_y at (i, j+1/2, n), J_z at (i, j, n+1/2)).  Since
  D . (D x A) = 0 identically, the correction leaves the discrete continuity
  equation of the filtered current untouched.
* Loss: mean over the loss region and the three components of
  ((J - J_target) / n_e)^2; Adam (Kingma & Ba 2015) on FP32 master weights.
* BF16 emulation (``quant=True``) rounds weights, network inputs and hidden
  activations to bfloat16 (round to nearest even) where the GPU kernels do,
  so both sides take the same quantisation decisions.

Array axes are (component/channel, zeta plane, y, x).  3-D only.
"""
import numpy as np

LAYERS = ((3, 16), (16, 32), (32, 16), (16, 3))
TAPS = [(dz, dy, dx) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]


def n_params():
    return sum(co * ci * 27 + co for ci, co in LAYERS)


def unpack(theta):
    """Flat parameter vector -> [(W (Cout, Cin, 3, 3, 3), b (Cout,)), ...],
    layer by layer, each W followed by its b."""
    out, k = [], 0
    for ci, co in LAYERS:
        W = np.asarray(theta[k:k + co * ci * 27], dtype=np.float64).reshape(co, ci, 3, 3, 3)
        k += co * ci * 27
        b = np.asarray(theta[k:k + co], dtype=np.float64)
        k += co
        out.append((W, b))
    return out


def pack(layers):
    return np.concatenate([np.concatenate([W.ravel(), b.ravel()]) for W, b in layers])


def bf16(a):
    """Round to bfloat16 (nearest, ties to even), via float32, returned as
    float64.  Finite inputs only."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def shift(x, dz, dy, dx):
    """out[..., z, y, x] = x[..., z + dz, y + dy, x + dx]; periodic in y and x,
    zero outside the stored planes in z."""
    out = np.roll(x, (-dy, -dx), axis=(-2, -1))
    if dz == 0:
        return out
    res = np.zeros_like(out)
    if dz > 0:
        res[..., :-dz, :, :] = out[..., dz:, :, :]
    else:
        res[..., -dz:, :, :] = out[..., :dz, :, :]
    return res


def conv3d(x, W, b):
    """x (Cin, Z, Y, X), W (Cout, Cin, 3, 3, 3), b (Cout,) -> (Cout, Z, Y, X)."""
    y = np.empty((W.shape[0],) + x.shape[1:])
    y[:] = b[:, None, None, None]
    for dz, dy, dx in TAPS:
        y += np.tensordot(W[:, :, dz + 1, dy + 1, dx + 1], shift(x, dz, dy, dx), axes=(1, 0))
    return y


def conv3d_backward(x, W, gy):
    """Gradients of sum(gy * conv3d(x, W, b)) with respect to x, W and b."""
    gx = np.zeros_like(x)
    gW = np.zeros_like(W)
    for dz, dy, dx in TAPS:
        gW[:, :, dz + 1, dy + 1, dx + 1] = np.tensordot(gy, shift(x, dz, dy, dx),
                                                        axes=([1, 2, 3], [1, 2, 3]))
        back = np.tensordot(W[:, :, dz + 1, dy + 1, dx + 1], gy, axes=(0, 0))
        gx += shift(back, -dz, -dy, -dx)
    return gx, gW, gy.sum(axis=(1, 2, 3))


def forward(theta, X, quant=False):
    """Network output A and the per-layer inputs (for the backward pass)."""
    layers = unpack(theta)
    h = bf16(X) if quant else X
    inputs = []
    for l, (W, b) in enumerate(layers):
        inputs.append(h)
        z = conv3d(h, bf16(W) if quant else W, b)
        if l < len(layers) - 1:
            h = np.maximum(z, 0.0)
            if quant:
                h = bf16(h)
        else:
            h = z
    return h, inputs


def backward(theta, inputs, gA, quant=False):
    """Parameter gradient (flat, same layout as theta) given dLoss/dA.
    Under ``quant`` the incoming gradient of every layer is rounded to bf16
    before it meets bf16 weights or activations, as in the GPU kernels."""
    layers = unpack(theta)
    grads = [None] * len(layers)
    g = gA
    for l in range(len(layers) - 1, -1, -1):
        W, b = layers[l]
        gq = bf16(g) if quant else g
        gx, gW, gb = conv3d_backward(inputs[l], bf16(W) if quant else W, gq)
        grads[l] = (gW, gb)
        if l > 0:
            g = gx * (inputs[l] > 0.0)
    return pack(grads)


# ---------------------------------------------------------------------------
# staggered curl and divergence (spacings hx, hy, h); arrays (Z, Y, X)

def _bz(a):   # a at plane n - 1 (zero below plane 0)
    return shift(a, -1, 0, 0)


def _fz(a):   # a at plane n + 1 (zero above the last plane)
    return shift(a, 1, 0, 0)


def curl(A, hx, hy, h):
    """D x A on the current's staggering, from A on cell faces."""
    Ax, Ay, Az = A
    cx = (Az - shift(Az, 0, -1, 0)) / hy - (Ay - _bz(Ay)) / h
    cy = (Ax - _bz(Ax)) / h - (Az - shift(Az, 0, 0, -1)) / hx
    cz = (Ay - shift(Ay, 0, 0, -1)) / hx - (Ax - shift(Ax, 0, -1, 0)) / hy
    return np.stack([cx, cy, cz])


def curl_adjoint(G, hx, hy, h):
    """Transpose of ``curl``: <G, curl(A)> = <curl_adjoint(G), A>."""
    gx, gy, gz = G
    ax = (gy - _fz(gy)) / h - (gz - shift(gz, 0, 1, 0)) / hy
    ay = -(gx - _fz(gx)) / h + (gz - shift(gz, 0, 0, 1)) / hx
    az = (gx - shift(gx, 0, 1, 0)) / hy - (gy - shift(gy, 0, 0, 1)) / hx
    return np.stack([ax, ay, az])


def divergence(J, hx, hy, h):
    """D . J at the nodes (backward differences of the staggered current)."""
    Jx, Jy, Jz = J
    return ((Jx - shift(Jx, 0, 0, -1)) / hx + (Jy - shift(Jy, 0, -1, 0)) / hy
            + (Jz - _bz(Jz)) / h)


def binomial(J, passes=1):
    """1-2-1 along x and y (periodic) and zeta (zero beyond the planes), per
    component, ``passes`` times."""
    out = np.array(J, dtype=np.float64)
    for _ in range(passes):
        for ax in (-1, -2):
            out = 0.25 * (np.roll(out, 1, axis=ax) + 2.0 * out + np.roll(out, -1, axis=ax))
        out = 0.25 * (_bz(out) + 2.0 * out + _fz(out))
    return out


# ---------------------------------------------------------------------------

def apply(theta, Jraw, n_e, hx, hy, h, passes=1, quant=False):
    """Denoised current F(J_raw) + s D x A(J_raw / n_e), s = n_e h.  Returns
    (J, A, filtered J, network inputs)."""
    A, inputs = forward(theta, np.asarray(Jraw) / n_e, quant)
    Jf = binomial(Jraw, passes)
    return Jf + (n_e * h) * curl(A, hx, hy, h), A, Jf, inputs


def loss_and_grad(theta, Jraw, Jtarget, n_e, hx, hy, h, region, passes=1, quant=False):
    """Loss mean(((J - J_target) / n_e)^2) over planes region = (lo, hi) of the
    three components, and its gradient with respect to theta."""
    J, A, _, inputs = apply(theta, Jraw, n_e, hx, hy, h, passes, quant)
    lo, hi = region
    mask = np.zeros(J.shape[1:])
    mask[lo:hi] = 1.0
    N = 3 * (hi - lo) * J.shape[2] * J.shape[3]
    r = (J - Jtarget) / n_e * mask
    loss = float(np.sum(r * r) / N)
    gJ = 2.0 * r / (n_e * N)
    gA = (n_e * h) * curl_adjoint(gJ, hx, hy, h)
    return loss, backward(theta, inputs, gA, quant)


def continuity_rel(J, Jf, hx, hy, h):
    """Residual test of the denoised current: ||D.(J - F(J_raw))|| over
    ||D.F(J_raw)||, i.e. the continuity residual the correction adds,
    relative to the size of the filtered current's divergence."""
    num = np.sqrt(np.sum(divergence(J - Jf, hx, hy, h) ** 2))
    den = np.sqrt(np.sum(divergence(Jf, hx, hy, h) ** 2))
    return num / den if den > 0 else (0.0 if num == 0 else np.inf)


def correction_ratio(J, Jf):
    """Size test of the denoised current: ||J - F(J_raw)|| over ||F(J_raw)||,
    the correction relative to the filtered current it corrects."""
    num = np.sqrt(np.sum((J - Jf) ** 2))
    den = np.sqrt(np.sum(Jf ** 2))
    return num / den if den > 0 else (0.0 if num == 0 else np.inf)


def keep_network(J, Jf, hx, hy, h, threshold, corr_max=1.0):
    """The step keeps the denoised current J when its continuity ratio is at
    most threshold and its correction is at most corr_max times the filtered
    current; otherwise it falls back to F(J_raw)."""
    return bool(continuity_rel(J, Jf, hx, hy, h) <= threshold and correction_ratio(J, Jf) <= corr_max)


def adam(theta, m, v, g, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """Adam step t (1-based) with bias correction; returns new (theta, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
