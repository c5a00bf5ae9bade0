"""Writes photoexcitation_sphere16.npy: the photoexcitation rates Gamma_PE
(s^-1 per atom in the lower level) that the oracle measures on the 16^3
sphere workload (10-level atom, 200 lines, 1e5 packets): every packet
transported from the cold-start populations, estimators summed per (cell,
line) and divided by n_l V (Sec. 2.3: rates from the estimators). The
positive values, sorted, are the table from which the batched three-stage
problem takes the photoexcitation rate of each radiative level pair, so that
its rate matrices carry rates the method itself produced.

Run from the repository root: python3 -m synth.make_photoexcitation_table
(calls the oracle only; the stored table is an input of both the library and
the oracle)."""
import os

import numpy as np

import oracle
import synth

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "photoexcitation_sphere16.npy")


def main():
    w = synth.sphere_small()
    inp = oracle.nlte_inputs_from_workload(w)
    pops = np.zeros((w.n_cells, w.atom.n_levels))
    for c in np.where(w.n_species > 0)[0]:
        pops[c] = oracle.nlte_cold(inp, int(c))
    r = oracle.transport(oracle.transport_inputs_from_workload(w))
    est = oracle.dense_estimator(r["records"], w.n_cells, w.n_lines)
    V = (2 * w.beta_max / w.n * synth.C_CGS * w.t_exp) ** 3
    gam = oracle.rates(est, pops, w.atom, V)
    table = np.sort(gam[gam > 0])
    np.save(OUT, table)
    print(f"{OUT}: {table.size} rates, {table[0]:.3e} .. {table[-1]:.3e} s^-1, "
          f"median {np.median(table):.3e}")


if __name__ == "__main__":
    main()
