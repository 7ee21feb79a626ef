"""Oracle for the nucleon correlators built from the solver's propagators.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Plain numpy, FP64,
written from the paper's definitions (von Hippel, Rae, Shintani, Wittig,
arXiv:1605.00564, section 2.3):

* the interpolating field N_alpha = eps^{abc} (u^a C gamma_5 d^b) u^c_alpha
  (eq. Nop) and its two-point function, obtained here by Wick's theorem;
* the sequential sources of the three-point functions (forward sink at t_s,
  backward sink at T - t_s with the opposite parity projector), as the
  derivative of the projected two-point contraction with respect to one
  quark line, carried to the sink side by gamma_5-hermiticity;
* the three-point function from the sequential propagators.

Conventions.  A propagator from a point source at x0 is the 12 solutions
x_j = M^{-1} delta_{x0} e_j of the library (j = 3 spin + colour), so
S(x)[s, c, s', c'] = x_{3 s' + c'}(x)[s, c] is M^{-1}(x, x0) (the mass-
normalised propagator is 2 kappa times it; no factor is applied).
C = gamma_0 gamma_2 (it satisfies C gamma_mu C^{-1} = -gamma_mu^T in the
operator's chiral basis), Gamma = C gamma_5, and the conjugate field is
Nbar_{alpha'} = eps^{a'b'c'} ubar^{c'}_{alpha'} (dbar^{b'} Gamma ubar^{a' T}).
Wick's theorem then gives, per sink site x, with U the u and D the d
propagator (both S for degenerate flavours) and Q^{bb'} = Gamma D^{bb'} Gamma:
    C_{alpha alpha'}(x) = eps_{abc} eps_{a'b'c'} [ U^{cc'}_{alpha alpha'} tr(Q^{bb'} U^{aa' T})
                                                   - (U^{ca'} Q^{bb' T} U^{ac'})_{alpha alpha'} ].
"""

from __future__ import annotations

import numpy as np

import synth


def levi_civita():
    e = np.zeros((3, 3, 3))
    for a, b, c, s in [(0, 1, 2, 1), (1, 2, 0, 1), (2, 0, 1, 1), (0, 2, 1, -1), (2, 1, 0, -1), (1, 0, 2, -1)]:
        e[a, b, c] = s
    return e


def charge_conjugation():
    """C = gamma_0 gamma_2 (chiral basis of the operator)."""
    from . import gamma_matrices
    g, _ = gamma_matrices()
    return g[0] @ g[2]


def cg5():
    from . import gamma_matrices
    g, _ = gamma_matrices()
    return charge_conjugation() @ g[4]


def propagator_matrix(prop):
    """prop[12, V, 4, 3] (solution j = 3 s' + c') -> S[V, s, c, s', c']."""
    V = prop.shape[1]
    return np.ascontiguousarray(prop.reshape(4, 3, V, 4, 3).transpose(2, 3, 4, 0, 1))


def contract(U1, U2, D):
    """C_{alpha alpha'}(x) [V, 4, 4] for propagator matrices [V, s, c, s', c'].
    U1 is the u line of the first factor of each Wick term (U^{cc'} in the
    first, U^{ca'} in the second), U2 the other (U^{aa'}, U^{ac'})."""
    eps = levi_civita()
    G = cg5()
    Q = np.einsum("bg,xgBhC,hd->xbBdC", G, D, G)        # Q^{BC}_{bd}: spin b, d; colours B, C
    # term 1: U1^{cc'} tr(Q^{bb'} U2^{aa' T}) = U1^{cc'}_{al al'} sum_{ss'} Q^{bb'}_{ss'} U2^{aa'}_{ss'}
    tr = np.einsum("xsbtB,xsatA->xabAB", Q, U2)           # [x, a, b, a', b']
    T = np.einsum("abc,ABC,xabAB->xcC", eps, eps, tr)     # [x, c, c']
    t1 = np.einsum("xcC,xicjC->xij", T, U1)
    # term 2: -(U1^{ca'} Q^{bb' T} U2^{ac'})_{al al'}
    t2 = np.einsum("abc,ABC,xicrA,xsbrB,xsajC->xij", eps, eps, U1, Q, U2)
    return t1 - t2


def timeslice_sum(Cx, dims, t0):
    """G[t] = sum over the sites of timeslice (t0 + t) mod T of Cx[x]."""
    T = dims[0]
    spatial = synth.volume(dims) // T
    per_t = Cx.reshape(T, spatial, *Cx.shape[1:]).sum(axis=1)
    return np.roll(per_t, -t0, axis=0)


def nucleon_2pt(prop, dims, t0):
    """G(t)_{alpha alpha'} [T, 4, 4] of the point source at time t0, zero momentum."""
    S = propagator_matrix(np.asarray(prop, np.complex128))
    return timeslice_sum(contract(S, S, S), dims, t0)


def project(G, P):
    """tr(P G(t)) for G[T, 4, 4]."""
    return np.einsum("ji,tij->t", P, G)


def parity_projectors():
    """P+ = (1 + gamma_0)/2 and P- = (1 - gamma_0)/2."""
    from . import gamma_matrices
    g, _ = gamma_matrices()
    return 0.5 * (np.eye(4) + g[0]), 0.5 * (np.eye(4) - g[0])


def sink_kernel(S, P, flavour):
    """K(x)[s, c, s', c'] = d tr(P C(x)) / d S_f(x)[s, c, s', c'] for flavour
    f = 'd' (one line) or 'u' (two lines), all propagators equal to S."""
    eps = levi_civita()
    G = cg5()
    Q = np.einsum("bg,xgBhC,hd->xbBdC", G, S, G)
    trPU = np.einsum("ji,xiajA->xaA", P, S)                      # tr(P S^{aa'}) [x, a, a']
    if flavour == "d":
        # d tr(P C) / d D^{bb'}_{gg'} =
        #   eps eps [ tr(P U^{cc'}) (G^T U^{aa'} G^T)_{gg'} - (G^T U^{ac'} P U^{ca'} G^T)_{gg'} ]
        GU = np.einsum("kg,xkalA,hl->xgahA", G, S, G)           # (G^T U^{aa'} G^T) [x, g, a, h, a']
        k1 = np.einsum("abc,ABC,xcC,xgahA->xgbhB", eps, eps, trPU, GU)
        Y = np.einsum("xiajC,jk,xkcmA->xaCicmA", S, P, S)         # (U^{ac'} P U^{ca'})_{im}
        k2 = np.einsum("abc,ABC,ig,xaCicmA,hm->xgbhB", eps, eps, G, Y, G)
        return k1 - k2
    # u: four occurrences
    # term 1, U^{cc'}: (P^T)_{gg'} tr(Q^{bb'} U^{aa' T})
    tr = np.einsum("xsbtB,xsatA->xabAB", Q, S)
    k = np.einsum("abc,ABC,xabAB,hg->xgchC", eps, eps, tr, P)
    # term 1, U^{aa'}: Q^{bb'}_{gg'} tr(P U^{cc'})
    k = k + np.einsum("abc,ABC,xcC,xgbhB->xgahA", eps, eps, trPU, Q)
    # term 2, U^{ca'}: -(P^T U^{ac' T} Q^{bb'})_{gg'}
    k = k - np.einsum("abc,ABC,kg,xmakC,xmbhB->xgchA", eps, eps, P, S, Q)
    # term 2, U^{ac'}: -(Q^{bb'} U^{ca' T} P^T)_{gg'}
    k = k - np.einsum("abc,ABC,xgbmB,xkcmA,hk->xgahC", eps, eps, Q, S, P)
    return k


def nucleon_seq_sources(prop, dims, t_sink, P, flavour):
    """The 12 sequential sources eta_j [12, V, 4, 3] for a sink on timeslice
    t_sink with projector P: eta_j(x)_i = gamma_5,ii conj(K(x)_{i j}) on
    t_sink, zero elsewhere; i = (s, c) at the sink, j = 3 s' + c' at the source."""
    from . import gamma_matrices
    g, _ = gamma_matrices()
    g5 = np.real(np.diag(g[4]))
    S = propagator_matrix(np.asarray(prop, np.complex128))
    V = S.shape[0]
    spatial = V // dims[0]
    sel = (np.arange(V) // spatial) == t_sink
    K = sink_kernel(S[sel], np.asarray(P, np.complex128), flavour)       # [n, s, c, s', c']
    eta = np.zeros((4, 3, V, 4, 3), np.complex128)                        # [s', c', x, s, c]
    eta[:, :, sel] = np.conj(K).transpose(3, 4, 0, 1, 2) * g5[None, None, None, :, None]
    return eta.reshape(12, V, 4, 3)


def nucleon_3pt(seqprop, prop, dims, t0, gamma_op):
    """sum over y on timeslice (t0 + t) mod T of sum_j (gamma_5 Sigma_j(y))^+
    Gamma_op x_j(y): the three-point function from the sequential
    propagators Sigma_j = M^{-1} eta_j and the forward solutions x_j."""
    from . import gamma_matrices
    g, _ = gamma_matrices()
    g5 = np.real(np.diag(g[4]))
    sig = np.asarray(seqprop, np.complex128) * g5[None, None, :, None]
    per = np.einsum("jxsc,st,jxtc->x", np.conj(sig), np.asarray(gamma_op, np.complex128),
                    np.asarray(prop, np.complex128))
    T = dims[0]
    return np.roll(per.reshape(T, -1).sum(axis=1), -t0)
