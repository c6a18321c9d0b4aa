"""Error bound of a forward-difference Jacobian column (test helper).

A forward difference (F(x + h e_j) - F(x)) / h carries a truncation error
of order h |d2F/dx_j2| and a rounding error of order eps S_r / h, where S_r
is the magnitude of the terms that cancel in F_r.  For mass-action kinetics
every rate term is homogeneous in the concentrations, so
S_r ~ sum_c |J_rc| |x_c| + |F_r| (J the exact Jacobian)."""
import numpy as np

EPS = 2.0 ** -52


def fd_steps(x, n_species):
    """The steps the finite-difference Jacobian takes (the representable
    difference of x_j and x_j + 2^-26 max(|x_j|, floor))."""
    x = np.asarray(x, float)
    floor = np.where(np.arange(x.shape[0]) < n_species, 1e-10, 1.0)
    d = 2.0 ** -26 * np.maximum(np.abs(x), floor)
    return (x + d) - x


def fd_bound(J_exact, F, x, h, rel, k_round, J_shift=None):
    """rel |J| + k_round eps S_r / h_j, plus, when J_shift is given (column j
    of the exact Jacobian at x + h_j e_j, [n][n]), the truncation bound
    |J_shift - J|: by the mean-value form the difference quotient is the
    average of column j of J over the step, which lies within that change
    where the column is monotone along the step."""
    S = np.abs(J_exact) @ np.abs(x) + np.abs(F)
    b = rel * np.abs(J_exact) + k_round * EPS * S[:, None] / h[None, :]
    if J_shift is not None:
        b = b + np.abs(J_shift - J_exact)
    return b


def shifted_columns(jac, x, h):
    """[n][n] whose column j is column j of jac(x + h_j e_j)."""
    n = x.shape[0]
    out = np.zeros((n, n))
    for j in range(n):
        xs = np.array(x, float)
        xs[j] = x[j] + h[j]
        out[:, j] = jac(xs)[:, j]
    return out


def within(diff, bound):
    diff = np.abs(diff)
    return bool(np.all((diff <= bound) | (diff == 0.0)))
