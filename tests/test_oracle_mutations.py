"""Strength of the oracle's surface-tension and time-step pins: each plausible
mistake below is planted in a temporary copy of the oracle (CPU only; the
repository's oracle is never modified) and the pins that cover that part must
then fail.  A pin that still passes with the mistake in place would not pin
anything."""

import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

# (oracle file, original text, planted text, what the mistake is)
MUTATIONS = [
    ("residual.py", "csf = prm.sigma * kappa * dG", "csf = -prm.sigma * kappa * dG", "flipped CSF force sign"),
    ("residual.py", "csf = prm.sigma * kappa * dG", "csf = prm.sigma * kappa", "delta_Gamma dropped"),
    ("residual.py", "ej = ej + csf * u[j] * nhat[j]", 'ej = ej + csf * u[j] * raw["gA"][j]',
     "u.grad alpha in place of u.n in the CSF work"),
    ("residual.py", "ej = ej + csf * u[j] * nhat[j]", "ej = ej", "CSF work dropped from the energy"),
    ("residual.py", "kappa = -sum(", "kappa = sum(", "curvature sign"),
    ("residual.py", "sj = sj + csf * nhat[j]", 'sj = sj + csf * raw["gA"][j]', "grad alpha in place of n"),
    ("residual.py", 'torch.sqrt((raw["gA"] * raw["gA"]).sum(0)', 'torch.sqrt((raw["gP"] * raw["gP"]).sum(0)',
     "delta_Gamma from the level set"),
    ("stepper.py", 'nu = max(nu, float((mu / pr["rho"]).max()))', "nu = max(nu, float(mu.max()))",
     "dynamic in place of kinematic viscosity"),
    ("stepper.py", 'nu = max(nu, float((mu / pr["rho"]).max()))', 'nu = nu + float((mu / pr["rho"]).max())',
     "sum in place of max"),
    ("stepper.py", "(mesh.p + 1) ** 2 * d * nu", "d * nu", "missing (p+1)^2 of the diffusive rate"),
    ("stepper.py", 'wave = torch.abs(pr["u"]).sum(0) + d * pr["c"]', 'wave = torch.abs(pr["u"]).sum(0) + pr["c"]',
     "missing d on the sound speed"),
]
PINS = "csf or viscous_branch or time_step_rule"


@pytest.fixture(scope="module")
def scratch(tmp_path_factory):
    dst = tmp_path_factory.mktemp("mutated")
    for d in ("oracle", "tests", "paper_2306_05002_amd"):
        shutil.copytree(os.path.join(ROOT, d), os.path.join(dst, d),
                        ignore=shutil.ignore_patterns("*.so", "_build", "__pycache__", "csrc"))
    return str(dst)


def _pins(cwd):
    r = subprocess.run([sys.executable, "-m", "pytest", "tests/test_oracle_pins.py", "-q", "-k", PINS,
                        "-p", "no:cacheprovider"], cwd=cwd, capture_output=True, text=True)
    return r.returncode, r.stdout.strip().splitlines()[-1] if r.stdout.strip() else r.stderr


def test_pins_pass_on_the_unmodified_copy(scratch):
    rc, last = _pins(scratch)
    assert rc == 0, last


@pytest.mark.parametrize("fname,orig,planted,what", MUTATIONS, ids=[m[3] for m in MUTATIONS])
def test_planted_mistake_fails_a_pin(scratch, fname, orig, planted, what):
    path = os.path.join(scratch, "oracle", fname)
    text = open(os.path.join(ROOT, "oracle", fname)).read()
    assert text.count(orig) >= 1, f"the oracle no longer contains {orig!r}"
    try:
        open(path, "w").write(text.replace(orig, planted, 1))
        rc, last = _pins(scratch)
    finally:
        open(path, "w").write(text)
    assert rc != 0, f"no pin failed with the mistake '{what}' planted ({last})"
