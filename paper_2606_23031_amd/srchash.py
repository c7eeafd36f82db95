"""Hash of the HIP sources, to tie stored counter measurements to the
kernels they were taken on."""
import glob
import hashlib
import os

HERE = os.path.dirname(os.path.abspath(__file__))


def csrc_hash():
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(HERE, "csrc", "*"))):
        with open(f, "rb") as fh:
            h.update(os.path.basename(f).encode())
            h.update(fh.read())
    return h.hexdigest()[:16]
