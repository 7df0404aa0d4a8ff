import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# The tests neither read nor write the user's pair-shape tuning cache; the
# cache's own tests point it at a temporary file.
os.environ["NFS_TUNE_CACHE"] = "off"


def pytest_configure(config):
    config.addinivalue_line(
        "markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
