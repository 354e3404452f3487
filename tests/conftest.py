import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: CPU test that takes more than a few seconds")


CARD_RANKS = {"A": 0, "2": 1, "3": 2, "4": 3, "5": 4, "6": 5, "7": 6, "8": 7, "9": 8,
              "10": 9, "J": 10, "Q": 11, "K": 12}
CARD_SUITS = {"C": 0, "D": 1, "H": 2, "S": 3}


def card_index(name: str) -> int:
    """'10D' -> 37: index = 4*rank + suit (figure 'Mapping Cards to Indices')."""
    return 4 * CARD_RANKS[name[:-1]] + CARD_SUITS[name[-1]]


def cards_of(field: str):
    if field == "-":
        return []
    return [card_index(x) for x in field.split(",")]


def read_rows(path):
    rows = []
    with open(path) as fh:
        for line in fh:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append(line.split())
    return rows


@pytest.fixture(scope="session")
def golden_dir():
    return os.path.join(ROOT, "tests", "golden")
