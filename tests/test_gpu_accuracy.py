"""Accuracy report of the HIP path against the oracle, per workload, in the
terms the paper uses (Sec. 3.2 and 3.3):

* the literal relative test of every source term (1e-10) and Jacobian entry
  (1e-8 with a 1e-20 floor): the largest relative error, the number of
  entries that fail it and their condition numbers kappa = b / (u |ref|),
  b the oracle's running error bound of the entry;
* E_X of dT/dt, dS/dt and dn/dt (Sec. 3.2, relative error norm with the
  1e-10 absolute and 1e-6 relative weights);
* E_C at C = 1e15 and 1e20 (Sec. 3.3, the filtered relative error of the
  Jacobian) and E_L (the LAPACK-style norm).

The states are the workloads' own (seeded; the 13-species one in full, the
others sampled from their full-size batches), evaluated in the launch shape
the autotuner picks for the sparse Jacobian.  Every comparison also passes
the parity gates.  With PJ_ACCURACY_REPORT set, the reports are written to
that path as JSON.
"""
import json
import os

import numpy as np
import pytest

import oracle
from oracle import gates
from paper_1809_01029_amd import synth
from conftest import workload_file

pytestmark = pytest.mark.gpu

CASES = [("ns13", "conp", 1024), ("ns13", "conv", 1024), ("ns53", "conp", 96), ("ns111", "conp", 96),
         ("ns111", "conv", 96), ("ns360", "conp", 24)]
_REPORTS = {}


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.fixture(scope="module")
def api(torch_cuda):
    from paper_1809_01029_amd import api as a
    return a


@pytest.mark.parametrize("name,form,n", CASES)
def test_accuracy_report(torch_cuda, api, name, form, n, mech_dir):
    torch = torch_cuda
    m, path = workload_file(name, mech_dir)
    w = synth.WORKLOADS[name]
    st = synth.make_states(m, min(w.n_states, 4096), w.state_seed, T_range=w.T_range, P_range_atm=w.P_range_atm)
    idx = np.arange(n) if n >= st["T"].shape[0] else np.sort(
        np.random.default_rng(31).choice(st["T"].shape[0], n, replace=False))
    st = {k: v[idx] for k, v in st.items()}
    x, p = synth.pack_state(st, form, "C")
    mech = api.load_mechanism(path)
    xs, ps = torch.from_numpy(x).cuda(), torch.from_numpy(p).cuda()
    api.autotune(mech, xs, ps, form, "C", mode="sparse", reps=1)
    d = torch.empty_like(xs)
    j = api.eval_jacobian_sparse(mech, xs, ps, form, "C", dstate=d)
    torch.cuda.synchronize()
    o = oracle.Oracle(path)
    f_o, f_b = o.source(x, p, form, bound=True)
    J_o, J_b = o.jacobian(x, p, form, bound=True)
    f_g = d.cpu().numpy()
    J_g = api.sparse_to_dense(mech, j.cpu().numpy(), "C")
    gates.check_source(f_g, f_o, f_b, f"{name} {form} source")
    gates.check_jac(J_g, J_o, J_b, f"{name} {form} Jacobian")
    rep = gates.accuracy_report(f_g, f_o, f_b, J_g, J_o, J_b)
    rep["states"] = int(n)
    rep["launch_shape"] = list(mech.launch_shape(1))
    print(f"accuracy {name} {form}: {json.dumps(rep)}", flush=True)
    _REPORTS[f"{name}_{form}"] = rep
    out = os.environ.get("PJ_ACCURACY_REPORT")
    if out:
        with open(out, "w") as fh:
            json.dump(_REPORTS, fh, indent=1, sort_keys=True)
