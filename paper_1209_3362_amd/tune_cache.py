"""Persistent cache of pair-kernel launch shapes chosen by the autotuner.

A JSON file maps a key of (GPU architecture, frame size, lag list, spectrum
storage type, accumulation) to the (modes, waves) shape of every lag group,
as nfs_tune_pairs chose them; a later plan with the same key applies them
through nfs_set_pair_shapes instead of timing every shape again.

Environment:
    NFS_TUNE_CACHE    path of the JSON file (default
                      ~/.cache/paper_1209_3362_amd/pair_shapes.json), or
                      "off" to neither read nor write it;
    NFS_TUNE_REFRESH  set to 1 to time again and overwrite cached entries.
Host-side bookkeeping only: no arithmetic of the analysis happens here.
"""
import hashlib
import json
import os

DEFAULT = os.path.join(os.path.expanduser("~"), ".cache", "paper_1209_3362_amd",
                       "pair_shapes.json")


def cache_path():
    """The cache file, or None when caching is switched off."""
    p = os.environ.get("NFS_TUNE_CACHE", DEFAULT)
    return None if p.strip().lower() in ("", "off", "0", "none") else p


def refresh():
    return os.environ.get("NFS_TUNE_REFRESH", "") not in ("", "0")


def cache_key(arch, n, lags, spec, accum):
    lag_hash = hashlib.sha1(",".join(str(int(t)) for t in lags).encode()).hexdigest()[:16]
    return f"{arch}|n={int(n)}|lags={len(lags)}:{lag_hash}|spec={spec}|accum={accum}"


def load(path):
    try:
        with open(path) as fh:
            data = json.load(fh)
    except (OSError, ValueError):
        return {}
    return data if isinstance(data, dict) else {}


def lookup(path, key):
    """Cached [(modes, waves), ...] for `key`, or None."""
    if path is None:
        return None
    entry = load(path).get(key)
    if not isinstance(entry, list):
        return None
    try:
        return [(int(m), int(w)) for m, w in entry]
    except (TypeError, ValueError):
        return None


def store(path, key, shapes):
    """Add or replace `key` (atomic rename; other keys are kept)."""
    if path is None:
        return
    data = load(path)
    data[key] = [[int(m), int(w)] for m, w in shapes]
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    tmp = f"{path}.{os.getpid()}.tmp"
    with open(tmp, "w") as fh:
        json.dump(data, fh, indent=1, sort_keys=True)
    os.replace(tmp, path)
