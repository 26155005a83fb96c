"""Plant plausible mistakes in copies of the oracle modules; some pin must fail for each.

Each mutation edits one line of an oracle module's source, executes the edited source
as a fresh module and swaps it into the pin module for the duration of the check.
"""
import importlib
import inspect
import sys
import types

import pytest

from tests import oracle_pins as P

# (module, attribute of oracle_pins holding it, old text, new text, what the mistake is)
MUTATIONS = [
    ("oracle.transform", "otr", "return np.exp(2j * np.pi * theta)", "return np.exp(-2j * np.pi * theta)",
     "wrong sign of the exponent"),
    ("oracle.transform", "otr", "out += c[:, :1]", "out += 0 * c[:, :1]", "dropped empty-set term"),
    ("oracle.transform", "otr", "acc += Y[:, a:b] @ E.conj()", "acc += Y[:, a:b] @ E", "adjoint without conjugate"),
    ("oracle.transform", "otr", "E = _phase_matrix(x[a:b][:, list(u)], ell)    # (chunk, G)",
     "E = _phase_matrix(x[a:b][:, list(u)[::-1]], ell)", "coordinates of a term swapped"),
    ("oracle.transform", "otr", "2j * np.pi * ell[:, pos] * c", "2j * np.pi * ell[:, pos - 1] * c",
     "gradient uses the wrong frequency component"),
    ("oracle.transform", "otr", "out += y[a:b] @ np.exp(-2j * np.pi * theta)",
     "out += y[a:b] @ np.exp(2j * np.pi * theta)", "selected adjoint entries without conjugate"),
    ("oracle.transform", "otr", "K = iset.full_frequencies()[np.asarray(idx)].astype(np.float64)",
     "K = iset.full_frequencies()[np.sort(np.asarray(idx))].astype(np.float64)",
     "selected adjoint entries returned in sorted instead of requested order"),
    ("oracle.transform", "otr", "for a in range(0, x.shape[0], _CHUNK):\n        b = min(x.shape[0], a + _CHUNK)\n        theta",
     "for a in range(0, x.shape[0] - 1, _CHUNK):\n        b = min(x.shape[0] - 1, a + _CHUNK)\n        theta",
     "selected adjoint entries drop the last node"),
    ("oracle.cosine", "ocos", "out *= np.sqrt(2.0) * np.cos(np.pi * np.outer(xu[:, j], ell[:, j].astype(np.float64)))",
     "out *= np.cos(np.pi * np.outer(xu[:, j], ell[:, j].astype(np.float64)))", "cosine basis without sqrt(2)"),
    ("oracle.cosine", "ocos", "out *= np.sqrt(2.0) * np.cos(np.pi * np.outer(xu[:, j], ell[:, j].astype(np.float64)))",
     "out *= np.sqrt(2.0) * np.cos(2 * np.pi * np.outer(xu[:, j], ell[:, j].astype(np.float64)))",
     "cosine basis of the full period"),
    ("oracle.cosine", "ocos", "return list(range(1, N))", "return list(range(0, N - 1))",
     "cosine group includes frequency 0"),
    ("oracle.cosine", "ocos", "out[:, sl] = Y.sum(axis=1, keepdims=True)", "out[:, sl] = Y.mean(axis=1, keepdims=True)",
     "cosine adjoint empty set averaged"),
    ("oracle.cosine", "ocos", "acc += Y[:, a:b] @ _basis_matrix(x[a:b][:, list(u)], iset.freqs[i])",
     "acc += Y[:, a:b] @ _basis_matrix(x[a:b][:, list(u)[::-1]], iset.freqs[i])", "cosine adjoint coordinates swapped"),
    ("oracle.cosine", "ocos", "A *= np.where(kj > 0, np.sqrt(2.0) * np.cos(np.pi * np.outer(x[:, j], kj)), 1.0)",
     "A *= np.where(kj > 0, np.sqrt(2.0) * np.cos(np.pi * np.outer(x[:, j], kj)), 0.0)",
     "cosine dense matrix zero on inactive coordinates"),
    ("oracle.index_set", "oidx", "[k for k in range(-N // 2, N // 2) if k != 0]",
     "[k for k in range(-N // 2 + 1, N // 2 + 1) if k != 0]", "band shifted by one"),
    ("oracle.index_set", "oidx", "out.extend(itertools.combinations(range(d), t))",
     "out.extend(sorted(itertools.combinations(range(d), t), reverse=True))", "term order reversed"),
    ("oracle.lsqr", "olsqr", "damp = np.sqrt(2.0 * lam)", "damp = np.sqrt(lam)", "damping without the factor 2"),
    ("oracle.lsqr", "olsqr", "rhobar = -c * alpha", "rhobar = c * alpha", "sign of rhobar"),
    ("oracle.lsqr", "olsqr", "s = 1.0 / np.sqrt(omega)", "s = 1.0 / omega", "weights applied as W^-1"),
    ("oracle.fista", "ofista", "x[sl] = zu / (1.0 + xi * wu)", "x[sl] = zu / (1.0 + 2.0 * xi * wu)",
     "Lemma's 2 xi used with the Theorem's xi"),
    ("oracle.fista", "ofista", "zero_level = np.sqrt(np.sum(np.abs(zu) ** 2 / wu))",
     "zero_level = np.sqrt(np.sum(np.abs(zu) ** 2 * wu))", "zero threshold with omega instead of 1/omega"),
    ("oracle.fista", "ofista", "h = f + ((t - 1.0) / t_next) * (f - f_prev)", "h = f + (t / t_next) * (f - f_prev)",
     "momentum coefficient"),
    ("oracle.fista", "ofista", "grad = rmatvec(Fh - y)", "grad = rmatvec(y - Fh)", "gradient sign"),
    ("oracle.sensitivity", "osens", "var = np.sum(e[..., 1:], axis=-1, keepdims=True)",
     "var = np.sum(e, axis=-1, keepdims=True)", "variance including the empty set"),
    ("oracle.sensitivity", "osens", "out[..., i] = np.sum(g.real ** 2 + g.imag ** 2, axis=-1)",
     "out[..., i] = np.sum(np.abs(g), axis=-1) ** 2", "term norm as the squared l1 norm"),
    ("oracle.sensitivity", "osens", "mask[c] = 1 if rho[where[u]] > eps[len(u) - 1] else 0",
     "mask[c] = 1 if rho[where[u]] >= eps[len(u) - 1] else 0", "threshold not strict"),
    ("oracle.sensitivity", "osens",
     "e2 = norm2 + np.sum(np.abs(fhat - exact) ** 2, axis=-1) - np.sum(np.abs(exact) ** 2, axis=-1)",
     "e2 = norm2 + np.sum(np.abs(fhat - exact) ** 2, axis=-1)", "error without the captured energy"),
    ("oracle.index_set", "oidx", "terms = [u for u, k in zip(terms, keep) if k or not u]",
     "terms = [u for u, k in zip(terms, keep) if k]", "subset drops the empty set"),
]


def _mutated(modname, old, new):
    mod = importlib.import_module(modname)
    src = inspect.getsource(mod)
    assert old in src, f"mutation anchor not found in {modname}: {old!r}"
    src = src.replace(old, new, 1)
    name = modname + "_mutant"
    m = types.ModuleType(name)
    m.__package__ = "oracle"
    sys.modules[name] = m          # dataclasses look their module up here
    try:
        exec(compile(src, name, "exec"), m.__dict__)
    finally:
        del sys.modules[name]
    return m


@pytest.mark.parametrize("modname,attr,old,new,what", MUTATIONS, ids=[m[4] for m in MUTATIONS])
def test_mutation_is_caught(monkeypatch, modname, attr, old, new, what):
    mutant = _mutated(modname, old, new)
    monkeypatch.setattr(P, attr, mutant)
    caught = []
    # pins that use the mutated module first (a pin that does not use it cannot catch it)
    order = sorted(P.PINS, key=lambda p: (attr + ".") not in inspect.getsource(p[1]))
    for name, fn, kw, tol in order:
        try:
            err = fn(**kw)
        except Exception:          # a crash also exposes the mistake
            caught.append(name)
            break
        if not err <= tol:
            caught.append(name)
            break
    assert caught, f"no pin caught: {what}"
