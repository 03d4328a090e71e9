"""Brute-force second quantisation on the Fock space of a few spinors, for
the oracle's pins: creation and annihilation operators as matrices (Jordan-
Wigner signs), determinants and operators built from them.  Spinors
0..o-1 are occupied in the reference, o..o+v-1 virtual."""
import itertools

import numpy as np


# Fock space of n spinors: basis |m>, m a bit mask, bit p = spinor p occupied.

def annihilator(n, p):
    dim = 1 << n
    a = np.zeros((dim, dim))
    for m in range(dim):
        if m >> p & 1:
            sign = (-1) ** bin(m & ((1 << p) - 1)).count("1")
            a[m ^ (1 << p), m] = sign
    return a


class Fock:
    def __init__(self, o, v):
        self.o, self.v, self.n = o, v, o + v
        self.a = [annihilator(self.n, p) for p in range(self.n)]
        self.c = [x.T.copy() for x in self.a]
        ref = np.zeros(1 << self.n)
        ref[0] = 1.0
        for p in reversed(range(o)):
            ref = self.c[p] @ ref
        self.ref = ref

    def vir(self, a):
        return self.o + a

    def double(self, i, j, a, b):
        """|ij->ab> = a+_a a+_b a_j a_i |ref>."""
        A, B = self.vir(a), self.vir(b)
        return self.c[A] @ (self.c[B] @ (self.a[j] @ (self.a[i] @ self.ref)))

    def single(self, i, a):
        return self.c[self.vir(a)] @ (self.a[i] @ self.ref)

    def t2_op(self, t):
        """T2 = 1/4 sum t_ij^ab a+_a a+_b a_j a_i."""
        o, v = self.o, self.v
        T = np.zeros((1 << self.n, 1 << self.n), np.complex128)
        for i, j, a, b in itertools.product(range(o), range(o), range(v), range(v)):
            if t[i, j, a, b] != 0:
                T += 0.25 * t[i, j, a, b] * (self.c[self.vir(a)] @ self.c[self.vir(b)]
                                             @ self.a[j] @ self.a[i])
        return T

    def one_body(self, M):
        """sum_pq M[p, q] a+_p a_q over all spinors."""
        A = np.zeros((1 << self.n, 1 << self.n), np.complex128)
        for p in range(self.n):
            for q in range(self.n):
                if M[p, q] != 0:
                    A += M[p, q] * (self.c[p] @ self.a[q])
        return A



    def two_body(self, Lfull):
        """V = 1/2 sum_{pqrs} <pq|rs> a+_p a+_q a_s a_r with
        <pq|rs> = sum_P L^P_pr L^P_qs over all spinors."""
        n = self.n
        g = np.einsum("Ppr,Pqs->pqrs", Lfull, Lfull)
        C2 = [[self.c[p] @ self.c[q] for q in range(n)] for p in range(n)]
        A2 = [[self.a[s] @ self.a[r] for r in range(n)] for s in range(n)]
        V = np.zeros((1 << n, 1 << n), np.complex128)
        for p, q, r, s in itertools.product(range(n), repeat=4):
            if g[p, q, r, s] != 0:
                V += 0.5 * g[p, q, r, s] * (C2[p][q] @ A2[s][r])
        return V
