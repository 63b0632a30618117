"""python -m paper_2312_07440_amd.gen: write the generated process sources."""
from . import generate

if __name__ == "__main__":
    for name, em in generate().items():
        print(name, em.counts, "amplitudes", em.n_amp, "flow terms", em.n_jterms)
