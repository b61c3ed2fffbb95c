"""Closed-form cases shared by the oracle pins and the GPU tests: networks
whose exact trajectories follow from the mathematics alone (no oracle, no
library), so both sides are checked against the same independent facts."""
import numpy as np

from paper_1906_03958_amd import workloads as W


def R4(z):
    """RK4 amplification polynomial (Taylor polynomial of e^z of degree 4)."""
    return 1 + z + z * z / 2 + z ** 3 / 6 + z ** 4 / 24


# Transmitter release T(V) = 1 / (1 + exp(-(V - V_p) / K_p)) has exact special
# values: T(V_p) = 1/2, T(V_p + K_p ln 3) = 3/4, T(V_p - K_p ln 3) = 1/4.
# Release midpoints and slopes per synapse type for these pins, distinct per
# row so that reading another type's row moves T as well (float32-exact).
RELEASE_VK = {W.ACH: (2.0, 5.0), W.GABA_A: (-10.0, 4.0), W.GABA_B: (-20.0, 8.0)}


def release_kinetics():
    k = W.DEFAULT_KINETICS.copy()
    for t, (vp, kp) in RELEASE_VK.items():
        k[t, 3], k[t, 4] = vp, kp
    return k


def clamped_release_network(v_clamp, syn_type):
    """Two cells, cell 0 presynaptic and clamped at v_clamp (passive, E_L =
    V0 = v_clamp, no current), cell 1 postsynaptic to it through one synapse
    of syn_type.  Returns (instance, kinetics row of that type as float64)."""
    vc = float(np.float32(v_clamp))
    net = W.uncoupled(np.zeros(2), np.full(2, vc),
                      params=dict(g_Na=0.0, g_K=0.0, g_L=0.3, E_L=vc)).net
    net.n_pn = 2 if syn_type == W.ACH else 0
    net.kinetics = release_kinetics()
    g = np.full((1, 1), 0.375, np.float32)
    net.pathways = [W.Pathway(syn_type, 0, 1, 1, 2, g, np.ones((1, 1), np.uint8))]
    inst = W.Instance(net, np.full(2, vc, np.float32), W.Stimulus(np.zeros(2, np.float32)))
    return inst, net.kinetics.astype(np.float64)[syn_type]


def release_points(syn_type):
    """(clamp voltage, exact T there, bound on |T(float32 V) - T|): T' = T (1 -
    T) / K_p <= 1/(4 K_p), times the float32 rounding of the clamp voltage."""
    vp, kp = RELEASE_VK[syn_type]
    out = []
    for v, t in ((vp, 0.5), (vp + kp * np.log(3.0), 0.75), (vp - kp * np.log(3.0), 0.25)):
        dv = abs(float(np.float32(v)) - v)
        out.append((v, t, dv / (4.0 * kp)))
    assert out[0][2] == 0.0                # V_p itself is exact: T = 1/2 exactly
    return out


def gate_closed_form(a, b, T, dt, n, s0=0.0):
    z = -(a * T + b) * dt
    sinf = a * T / (a * T + b)
    return sinf + R4(z) ** np.arange(1, n + 1) * (s0 - sinf)


def slow_gaba_half_closed_form(k, dt, n):
    """(r, G) after 1..n RK4 steps from 0 at T_B = 1/2: the linear system y' =
    A y + c, A = [[-(r1/2 + r2), 0], [r3, -r4]], c = (r1/2, 0); one step maps
    y - y* by R(dt A)."""
    r1, r2, r3, r4 = k[5], k[6], k[7], k[8]
    A = np.array([[-(r1 * 0.5 + r2), 0.0], [r3, -r4]])
    c = np.array([r1 * 0.5, 0.0])
    ystar = -np.linalg.solve(A, c)
    M = dt * A
    Rm = np.eye(2) + M + M @ M / 2 + M @ M @ M / 6 + M @ M @ M @ M / 24
    cur, out = np.zeros(2), []
    for _ in range(n):
        cur = ystar + Rm @ (cur - ystar)
        out.append(cur.copy())
    return np.array(out)
