"""Oracle (test infrastructure only): coefficient tables of the time integrators
of Section 4 (the paper names the schemes but prints no coefficients).

ROW schemes are used in the transformed form of eq. Rosenbrock_General:
  (I/(gamma dt) - dR/dq) Y_i = R(q^n + sum_{j<i} a_ij Y_j) + (1/dt) sum_{j<i} c_ij Y_j,
  q^{n+1} = q^n + sum_j m_j Y_j.
A table published in the standard form (alpha_ij, gamma_ij, b_i) converts with
Gamma = (gamma_ij) lower triangular:  A = alpha Gamma^{-1},
C = diag(1/gamma) - Gamma^{-1},  m^T = b^T Gamma^{-1}  (Hairer & Wanner II, IV.7).

* ROW3 = ROS34PW2 (Rang & Angermann 2005), standard form as published.
* ROW4 = RODASP (Steinebach 1995), transformed form as published.
* ROW2: the coefficients of ROS2PR (Rang 2014) are not available here; a
  3-stage, order-2, stiffly accurate, L-stable ROW scheme with gamma = 1/4 is
  used in its place (b = (5/8, 1/8, 1/4), beta_21 = 1/2, alpha_21 = 1/2,
  alpha_31 = alpha_32 = 1/2).

ESDIRK schemes (eq. ESDIRK2: explicit first stage, a_ii = omega for i >= 2):
* ESDIRK2: 3 stages, gamma = 1 - 1/sqrt(2), c = (0, 2 gamma, 1), stiffly accurate.
* ESDIRK3 = ARK3(2)4L[2]SA implicit part (Kennedy & Carpenter), as used by Bijl et al.
* ESDIRK4 = ARK4(3)6L[2]SA implicit part (Kennedy & Carpenter), as used by Bijl et al.
"""
from __future__ import annotations

import math

import numpy as np


class RowTable:
    def __init__(self, name, gamma, A, C, m):
        self.name = name
        self.gamma = float(gamma)
        self.A = np.asarray(A, dtype=np.float64)
        self.C = np.asarray(C, dtype=np.float64)
        self.m = np.asarray(m, dtype=np.float64)
        self.s = len(self.m)

    @staticmethod
    def from_standard(name, alpha, gam, b):
        alpha = np.asarray(alpha, dtype=np.float64)
        gam = np.asarray(gam, dtype=np.float64)
        Ginv = np.linalg.inv(gam)
        g = gam[0, 0]
        A = alpha @ Ginv
        C = np.diag(1.0 / np.diag(gam)) - Ginv
        m = np.asarray(b, dtype=np.float64) @ Ginv
        return RowTable(name, g, np.tril(A, -1), np.tril(C, -1), m)

    def standard(self):
        """(alpha, Gamma, b) recovered from the transformed coefficients."""
        Ginv = np.diag(np.full(self.s, 1.0 / self.gamma)) - self.C
        Gam = np.linalg.inv(Ginv)
        return self.A @ Gam, Gam, self.m @ Gam


def _row2():
    g = 0.25
    alpha = np.zeros((3, 3))
    alpha[1, 0] = 0.5
    alpha[2, 0] = 0.5
    alpha[2, 1] = 0.5
    b = np.array([5 / 8, 1 / 8, 1 / 4])
    beta = np.zeros((3, 3))
    beta[1, 0] = 0.5
    beta[2, :] = b
    gam = beta - alpha
    np.fill_diagonal(gam, g)
    return RowTable.from_standard("ROW2", alpha, gam, b)


def _ros34pw2():
    g = 0.4358665215084590
    alpha = np.zeros((4, 4))
    gam = np.zeros((4, 4))
    alpha[1, 0] = 0.87173304301691801
    alpha[2, 0] = 0.84457060015369423
    alpha[2, 1] = -0.11299064236484185
    alpha[3, 2] = 1.0
    gam[1, 0] = -0.87173304301691801
    gam[2, 0] = -0.90338057013044082
    gam[2, 1] = 0.054180672388095326
    gam[3, 0] = 0.24212380706095346
    gam[3, 1] = -1.2232505839045147
    gam[3, 2] = 0.54526025533510214
    np.fill_diagonal(gam, g)
    b = np.array([0.24212380706095346, -1.2232505839045147, 1.5452602553351020, 0.43586652150845900])
    return RowTable.from_standard("ROW3", alpha, gam, b)


def _rodasp():
    A = np.zeros((6, 6))
    C = np.zeros((6, 6))
    A[1, 0] = 3.0
    A[2, :2] = [1.831036793486759, 0.4955183967433795]
    A[3, :3] = [2.304376582692669, -0.05249275245743001, -1.176798761832782]
    A[4, :4] = [-7.170454962423024, -4.741636671481785, -16.31002631330971, -1.062004044111401]
    A[5, :5] = [-7.170454962423024, -4.741636671481785, -16.31002631330971, -1.062004044111401, 1.0]
    C[1, 0] = -12.0
    C[2, :2] = [-8.791795173947035, -2.207865586973518]
    C[3, :3] = [10.81793056857153, 6.780270611428266, 19.53485944642410]
    C[4, :4] = [34.19095006749676, 15.49671153725963, 54.74760875964130, 14.16005392148534]
    C[5, :5] = [34.62605830930532, 15.30084976114473, 56.99955578662667, 18.40807009793095, -5.714285714285717]
    m = [-7.170454962423024, -4.741636671481785, -16.31002631330971, -1.062004044111401, 1.0, 1.0]
    return RowTable("ROW4", 0.25, A, C, m)


class EsdirkTable:
    def __init__(self, name, A, b):
        self.name = name
        self.A = np.asarray(A, dtype=np.float64)
        self.b = np.asarray(b, dtype=np.float64)
        self.c = self.A.sum(axis=1)
        self.s = len(self.b)
        self.gamma = float(self.A[1, 1])


def _esdirk2():
    g = 1.0 - 1.0 / math.sqrt(2.0)
    A = np.array([[0.0, 0.0, 0.0], [g, g, 0.0], [(1 - g) / 2, (1 - g) / 2, g]])
    return EsdirkTable("ESDIRK2", A, A[2])


def _esdirk3():
    g = 1767732205903 / 4055673282236
    A = np.array([
        [0.0, 0.0, 0.0, 0.0],
        [g, g, 0.0, 0.0],
        [2746238789719 / 10658868560708, -640167445237 / 6845629431997, g, 0.0],
        [1471266399579 / 7840856788654, -4482444167858 / 7529755066697, 11266239266428 / 11593286722821, g]])
    return EsdirkTable("ESDIRK3", A, A[3])


def _esdirk4():
    g = 0.25
    A = np.zeros((6, 6))
    A[1, :2] = [g, g]
    A[2, :3] = [8611 / 62500, -1743 / 31250, g]
    A[3, :4] = [5012029 / 34652500, -654441 / 2922500, 174375 / 388108, g]
    A[4, :5] = [15267082809 / 155376265600, -71443401 / 120774400, 730878875 / 902184768, 2285395 / 8070912, g]
    A[5, :6] = [82889 / 524892, 0.0, 15625 / 83664, 69875 / 102672, -2260 / 8211, g]
    return EsdirkTable("ESDIRK4", A, A[5])


ROW = {"ROW2": _row2(), "ROW3": _ros34pw2(), "ROW4": _rodasp()}
ESDIRK = {"ESDIRK2": _esdirk2(), "ESDIRK3": _esdirk3(), "ESDIRK4": _esdirk4()}
