"""The committed l-predictor (trained on 200k generated spectra by the
device kernels; paper_2505_16932_amd/predictor_T5.{npy,json}) at work.

* A materialised subset: 2048 matrices U diag(sigma) V^T (Haar factors, the
  training families, s <= 256 and L <= 1024) run through learned plans; their GPU
  features against the oracle's features of the spectrum that LAPACK's SVD
  (numpy) finds in the bf16 input, the labels from that spectrum against the
  labels of the construction spectrum, the mean step count, and each GPU
  result's polar error (against that input's own polar factor U V^T from the
  same SVD) against the error Appendix C predicts for its chosen class.
* The GPT-small-shaped batch (48 matrices, sigma_i = 1/i) with selection and
  the fallback: no matrix ends with a larger polar error than under the fixed
  schedule (beyond 1%), per matrix reported with its class and steps.
"""
import numpy as np
import pytest

import synth
from oracle import mlp as OM
from tests.gpu_util import device_input, oracle_schedule, polar_error, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pe():
    import paper_2505_16932_amd as pe
    pe.lib()
    return pe


@pytest.fixture(scope="module")
def predictor(pe):
    params, meta = pe.load_predictor(T=5)
    assert meta["samples"] >= 200000 and meta["trained_with"].startswith("pe_mlp_train_step")
    assert [tuple(c) for c in meta["classes"]] == [tuple(c) for c in OM.CLASS_TABLE]
    return params


def test_materialised_subset(pe, predictor):
    import torch
    from paper_2505_16932_amd import learned as PL
    rng = np.random.Generator(np.random.PCG64(4242))
    abc4 = oracle_schedule(5)
    steps = OM.class_steps(5)
    scheds = OM.class_schedules(5)
    rows = []
    for batch in range(8):
        Gs, infos = [], []
        for k in range(256):
            while True:
                m_, n_, sig, fam = PL.sample_spectrum(rng)
                if max(m_, n_) <= 1024 and min(m_, n_) <= 256:
                    break
            S = synth.usv(rng, m_, n_, sig)
            g, v = device_input(S.G, torch.bfloat16)
            Gs.append(g)
            infos.append((S, v, sig))
        plan = pe.Plan(Gs, T=5, abc=abc4, compute="bf16", predictor=predictor, out_dtype=torch.float32)
        plan.launch(graph=False)
        torch.cuda.synchronize()
        cls, feats, _, _ = plan.selection()
        for k, (S, v, sig) in enumerate(infos):
            # the polar factor and spectrum of the values the device received
            # (bf16 rounding moves the singular vectors of the small singular
            # values, so the construction's U V^T is not that input's polar factor)
            Uv, sv, Vtv = np.linalg.svd(v, full_matrices=False)
            sh_svd = sv / (1.01 * np.linalg.norm(v) + 1e-7)
            f_svd = OM.features(min(v.shape), max(v.shape), OM.moments_from_spectrum(sh_svd))
            e_svd = OM.class_errors(sh_svd, 5, scheds)
            lab_svd = OM.label(e_svd, steps)
            sh_con = sig / (1.01 * np.linalg.norm(sig) + 1e-7)
            lab_con = OM.label(OM.class_errors(sh_con, 5, scheds), steps)
            perr = polar_error(to_np(plan.outs[k]), Uv @ Vtv)
            rows.append((np.abs(feats[k] - f_svd).max(), lab_svd == lab_con, steps[cls[k]],
                         e_svd[cls[k]], e_svd[OM.FIXED_CLASS], perr))
        plan.close()
    ferr = np.array([r[0] for r in rows])
    agree = np.mean([r[1] for r in rows])
    st = np.array([r[2] for r in rows])
    chosen, fixed = np.array([r[3] for r in rows]), np.array([r[4] for r in rows])
    perr = np.array([r[5] for r in rows])
    print(f"[predictor] {len(rows)} materialised matrices: max feature err {ferr.max():.2e}, "
          f"labels SVD vs construction agree {agree:.1%}, mean steps {st.mean():.2f}/5, "
          f"mean error chosen {chosen.mean():.4f} fixed {fixed.mean():.4f}, "
          f"worse on {np.mean(chosen > fixed * 1.001 + 1e-9):.1%}", flush=True)
    assert ferr.max() <= 2e-2
    assert agree >= 0.95
    assert st.mean() < 4.8
    # the GPU result's polar error is the predicted error of its class
    # (Appendix C), up to the bf16 path's own error
    gap = np.abs(perr - chosen) - (0.03 + 0.05 * chosen)
    for k in np.argsort(gap)[::-1][:5]:
        print(f"[predictor] matrix {k}: polar error {perr[k]:.4f}, predicted {chosen[k]:.4f}", flush=True)
    assert np.all(gap <= 0)


def test_gpt_small_batch_no_regression(pe, predictor):
    import torch
    mats = synth.gpt_small_batch()
    Gs = []
    for S in mats:
        g, _ = device_input(S.G, torch.bfloat16)
        Gs.append(g)
    abc4 = oracle_schedule(5)
    plan = pe.Plan(Gs, T=5, abc=abc4, compute="bf16", predictor=predictor, fallback_tau=0.45,
                   out_dtype=torch.float32)
    plan.launch(graph=True)
    torch.cuda.synchronize()
    cls, _, est, flags = plan.selection()
    fixed = pe.polar_batched(Gs, T=5, abc=abc4, compute="bf16", out_dtype=torch.float32)
    torch.cuda.synchronize()
    steps = OM.class_steps(5)
    worst = 0.0
    for k, S in enumerate(mats):
        P = S.polar()
        e_l = polar_error(to_np(plan.outs[k]), P)
        e_f = polar_error(to_np(fixed[k]), P)
        if k < 8 or e_l > e_f * 1.01:
            print(f"[predictor] gpt-small {k} {S.G.shape}: class {cls[k]} ({steps[cls[k]]} steps) "
                  f"flag {flags[k]} est {est[k]:.3f}  ||X-UV^T||_2 learned {e_l:.4f} fixed {e_f:.4f}",
                  flush=True)
        worst = max(worst, e_l / e_f)
    print(f"[predictor] gpt-small: classes {np.bincount(cls, minlength=8).tolist()}, "
          f"fallbacks {int(flags.sum())}, worst ratio learned/fixed {worst:.4f}", flush=True)
    assert worst <= 1.01
    plan.close()
